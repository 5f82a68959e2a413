// Learned closure: features of the coarse (nside 1) solution, a 4-layer MLP in
// BF16 on the matrix cores with FP32 accumulation (forward, backward, Adam),
// and the closure/fallback assembly.
//
// Network: h1 = silu(x W1 + b1), h2 = silu(h1 W2 + b2), h3 = silu(h2 W3 + b3),
// y = h3 W4 + b4; x has 16 inputs (12 features, 4 zero), hidden width 256,
// y = (m, s): m predicts log(J_fine/J_coarse), s the log variance of its error.
// Parameters live as FP32 master weights (layout W1[16][256], b1, W2[256][256],
// b2, W3[256][256], b3, W4[256][2], b4); BF16 copies are published after every
// update: transposed [N][K] for the forward products and [K][N] for the
// backward ones.
//
// Rounding points (mirrored by the FP64 reference in the tests): x, weights,
// stored pre-activations z and activations h = silu(z) are BF16; products
// accumulate in FP32 (MFMA); biases and the head are FP32; the backward signal
// dz = dh * silu'(z) is rounded to BF16 before it enters the matrix cores.
//
// Tiles: forward, one workgroup (4 waves) takes 64 or 128 samples, each wave
// owning 64 of the 256 output columns (v_mfma_f32_16x16x16_bf16), activations
// kept in LDS between layers; for many samples a persistent kernel holds the
// hidden weights in registers (v_mfma_f32_16x16x32_bf16).  Backward: a signal
// pass per 32-sample tile and a split-K weight pass over sample chunks, both on
// v_mfma_f32_16x16x32_bf16, then an ordered sum of the partials (deterministic).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "rt_internal.h"

namespace rt {

namespace {

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

constexpr int DIN = 16;
constexpr int HW = 256;   // hidden width
constexpr int DOUT = 2;
constexpr int LDH = HW + 8;  // LDS row stride (bf16 elements) of activation tiles
constexpr int LDX = DIN + 4;

// master-parameter offsets
constexpr int64_t OFF_W1 = 0;
constexpr int64_t OFF_B1 = OFF_W1 + DIN * HW;
constexpr int64_t OFF_W2 = OFF_B1 + HW;
constexpr int64_t OFF_B2 = OFF_W2 + HW * HW;
constexpr int64_t OFF_W3 = OFF_B2 + HW;
constexpr int64_t OFF_B3 = OFF_W3 + HW * HW;
constexpr int64_t OFF_W4 = OFF_B3 + HW;
constexpr int64_t OFF_B4 = OFF_W4 + HW * DOUT;
constexpr int64_t NPARAM = OFF_B4 + DOUT;
static_assert(NPARAM == RT_MLP_NPARAM, "parameter count");
constexpr int64_t MAX_SAMPLES = ((int64_t)1 << 31) - 1;  // sample indices are int32

// BF16 copies: forward (transposed [N][K]) and backward ([K][N]) layouts
constexpr int64_t WT1 = 0;                 // [256][16]
constexpr int64_t WT2 = WT1 + HW * DIN;    // [256][256]
constexpr int64_t WT3 = WT2 + HW * HW;     // [256][256]
constexpr int64_t WT4 = WT3 + HW * HW;     // [16][256], rows >= 2 zero
constexpr int64_t NWT = WT4 + 16 * HW;
constexpr int64_t WB2 = 0;                 // [256][256]
constexpr int64_t WB3 = WB2 + HW * HW;
constexpr int64_t NWB = WB3 + HW * HW;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16, round to nearest even (the hardware conversion)
__device__ inline uint16_t f2bf(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline uint32_t f2bf2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
__device__ inline float bf2f(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }
__device__ inline float bf_lo(uint32_t v) { return __builtin_bit_cast(float, v << 16); }
__device__ inline float bf_hi(uint32_t v) { return __builtin_bit_cast(float, v & 0xFFFF0000u); }
// x rounded to BF16 and read back as FP32: one conversion that puts bf16(x) in the high half
// and bf16(0) = 0 in the low half
__device__ inline float bfr(float x) { return __builtin_bit_cast(float, f2bf2(0.f, x)); }
// logistic function with the hardware reciprocal; silu(z) = z sigma(z)
__device__ inline float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigm(z); }
__device__ inline float dsilu(float z) {
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}

__device__ inline v4i16 ld4(const uint16_t* p) {  // 4 consecutive bf16 (8-byte aligned)
    return *(const v4i16*)p;
}
__device__ inline v4i16 pack4(uint16_t a, uint16_t b, uint16_t c, uint16_t d) {
    v4i16 r;
    r[0] = (short)a;
    r[1] = (short)b;
    r[2] = (short)c;
    r[3] = (short)d;
    return r;
}
__device__ inline v4f32 mfma(v4i16 a, v4i16 b, v4f32 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- publish / init

__global__ void k_publish(const float* __restrict__ w, uint16_t* __restrict__ wt, uint16_t* __restrict__ wb) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < HW * DIN) {  // W1t[n][k] = W1[k][n]
        const int n = (int)(i / DIN), k = (int)(i % DIN);
        wt[WT1 + i] = f2bf(w[OFF_W1 + (int64_t)k * HW + n]);
    }
    if (i < HW * HW) {
        const int n = (int)(i / HW), k = (int)(i % HW);
        wt[WT2 + i] = f2bf(w[OFF_W2 + (int64_t)k * HW + n]);
        wt[WT3 + i] = f2bf(w[OFF_W3 + (int64_t)k * HW + n]);
        wb[WB2 + i] = f2bf(w[OFF_W2 + i]);
        wb[WB3 + i] = f2bf(w[OFF_W3 + i]);
    }
    if (i < 16 * HW) {  // W4t[c][k] = W4[k][c], c < 2
        const int c = (int)(i / HW), k = (int)(i % HW);
        wt[WT4 + i] = c < DOUT ? f2bf(w[OFF_W4 + (int64_t)k * DOUT + c]) : (uint16_t)0;
    }
}

// ---------------------------------------------------------------- forward

// out[m][n] = bf16(silu(z)), z = bf16(b[n] + sum_k in[m][k] W[k][n]) for the
// 16*MTW samples m of the tile, W given as Wt[256][K].  The product is formed
// transposed (Z^T = Wt in^T: weights as the A operand, samples as B) so that a
// lane's four accumulators are four consecutive n of one sample and go out as
// one 8-byte store; they start from the bias.  Wave w owns n in [64w, 64w+64).
template <int MTW, int K, int ldin, bool KEEP>
__device__ __attribute__((always_inline)) inline void fwd_layer(const uint16_t* in, const uint16_t* __restrict__ Wt,
                                                                const float* __restrict__ bias, uint16_t* out,
                                                                uint16_t* __restrict__ zout, int64_t row0,
                                                                int nvalid) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    v4f32 acc[4][MTW];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float4 bb = *(const float4*)(bias + 64 * w + 16 * nt + 4 * g);
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) acc[nt][mt] = (v4f32){bb.x, bb.y, bb.z, bb.w};
    }
    for (int k0 = 0; k0 < K; k0 += 16) {
        v4i16 a[4], b[MTW];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) a[nt] = ld4(Wt + (int64_t)(64 * w + 16 * nt + r) * K + k0 + 4 * g);
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) b[mt] = ld4(in + (mt * 16 + r) * ldin + k0 + 4 * g);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int mt = 0; mt < MTW; ++mt) acc[nt][mt] = mfma(a[nt], b[mt], acc[nt][mt]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int n0 = 64 * w + 16 * nt + 4 * g;
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
            const int m = mt * 16 + r;
            const v4f32& a = acc[nt][mt];
            const uint32_t h01 = f2bf2(silu(bfr(a[0])), silu(bfr(a[1])));
            const uint32_t h23 = f2bf2(silu(bfr(a[2])), silu(bfr(a[3])));
            *(uint2*)(out + m * LDH + n0) = make_uint2(h01, h23);
            if (KEEP && m < nvalid)
                *(uint2*)(zout + (row0 + m) * HW + n0) = make_uint2(f2bf2(a[0], a[1]), f2bf2(a[2], a[3]));
        }
    }
}

// Forward over tiles of 16*MTW samples (rows[i] selects the input row of
// sample i when given); KEEP stores the BF16 pre-activations Z[3][n][256].
template <bool KEEP, int MTW>
__global__ __launch_bounds__(256, MTW == 4 ? 2 : 1) void k_mlp_fwd(
    const uint16_t* __restrict__ wt, const float* __restrict__ w, const uint16_t* __restrict__ X,
    const int32_t* __restrict__ rows, int64_t n, float* __restrict__ Y, uint16_t* __restrict__ Z) {
    constexpr int TS = 16 * MTW;
    __shared__ __attribute__((aligned(16))) uint16_t sx[TS * LDX];
    __shared__ __attribute__((aligned(16))) uint16_t sa[TS * LDH];
    __shared__ __attribute__((aligned(16))) uint16_t sb[TS * LDH];
    const int64_t row0 = (int64_t)blockIdx.x * TS;
    const int nvalid = (int)(n - row0 < TS ? n - row0 : TS);
    for (int t = threadIdx.x; t < TS * 4; t += 256) {  // TS x 16 inputs, 4 per thread
        const int m = t >> 2, q = t & 3;
        v4i16 v = (v4i16){0, 0, 0, 0};
        if (m < nvalid) {
            const int64_t src = rows ? (int64_t)rows[row0 + m] : row0 + m;
            v = ld4(X + src * DIN + 4 * q);
        }
        *(v4i16*)(sx + m * LDX + 4 * q) = v;
    }
    __syncthreads();
    uint16_t* Z1 = KEEP ? Z : nullptr;
    uint16_t* Z2 = KEEP ? Z + n * HW : nullptr;
    uint16_t* Z3 = KEEP ? Z + 2 * n * HW : nullptr;
    fwd_layer<MTW, DIN, LDX, KEEP>(sx, wt + WT1, w + OFF_B1, sa, Z1, row0, nvalid);
    __syncthreads();
    fwd_layer<MTW, HW, LDH, KEEP>(sa, wt + WT2, w + OFF_B2, sb, Z2, row0, nvalid);
    __syncthreads();
    fwd_layer<MTW, HW, LDH, KEEP>(sb, wt + WT3, w + OFF_B3, sa, Z3, row0, nvalid);
    __syncthreads();
    // head, transposed as the hidden layers: wave w takes the 16-sample groups
    // w, w+4, ...; the A operand is W4t (rows 0 and 1 used), so lanes with
    // g = 0 hold y[m][0..1]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    for (int grp = wv; grp < MTW; grp += 4) {
        v4f32 acc = (v4f32){0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < HW; k0 += 16)
            acc = mfma(ld4(wt + WT4 + (int64_t)r * HW + k0 + 4 * g), ld4(sa + (16 * grp + r) * LDH + k0 + 4 * g),
                       acc);
        const int m = 16 * grp + r;
        if (g == 0 && m < nvalid)
            *(float2*)(Y + (row0 + m) * DOUT) = make_float2(acc[0] + w[OFF_B4], acc[1] + w[OFF_B4 + 1]);
    }
}

// ---------------------------------------------------------------- forward, weights held in registers
//
// For inference over many samples: a persistent workgroup of 8 waves per CU
// loads the hidden layers' weights once and keeps them in registers, then
// streams tiles of 64 samples through all layers with the activations in LDS.
// Wave w owns the hidden columns [32w, 32w+32) of every layer: its strips of
// W2 and W3 (32 columns x 256 rows each) are A operands of
// v_mfma_f32_16x16x32_bf16, lane (r, g) holding row n0 + r, columns
// 32 ks + 8g .. +7 of Wt.  The activations are the B operands, lane (r, g)
// reading 16 contiguous bytes of sample m0 + r; the four accumulators of a
// lane are four consecutive columns of one sample (one 8-byte LDS store).
// The first layer (K = 16, padded to 32 with zeros) and the head read their
// weights from LDS.  Rounding points and results are those of k_mlp_fwd (the
// products are summed 32 at a time instead of 16, so a BF16 rounding of z may
// fall the other way).
typedef short v8i16 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int PT = 64;          // samples per tile
constexpr int PWAVES = 8;       // waves per workgroup
constexpr int LDP = HW + 8;     // LDS row stride (bf16) of activation tiles
constexpr int LDXP = 32 + 8;    // LDS row stride of the input tile (K padded to 32)
constexpr int LDW1 = 32 + 8;    // LDS row stride of W1t (K padded to 32)
constexpr int64_t WS_MIN_SAMPLES = 65536;  // below this the per-tile kernel (k_mlp_fwd) fills the chip better

__device__ inline v4f32 mfma32(v8i16 a, v8i16 b, v4f32 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}
__device__ inline v8i16 ld8(const uint16_t* p) { return *(const v8i16*)p; }  // 16-byte aligned

// Each tile is taken in two halves of 32 samples, A and B, one half behind
// the other: while a wave's matrix products of one half run, its epilogue
// (BF16 z, SiLU, BF16 h) of the other half's previous layer is issued
// between them, so the matrix cores and the vector ALUs work at the same time
// instead of in turns between the layer barriers.  Phases of a tile (each
// ends at a barrier; M = products, E = epilogue, layer 1..3):
//   M(B,1)+E(A,1), M(A,2)+E(B,1), M(B,2)+E(A,2), M(A,3)+E(B,2), M(B,3)+E(A,3),
//   E(B,3) with the next tile's input load, then the head of this tile with
//   M(A,1) of the next.  Layer l's activations go to ha (l odd) or hb (l even),
//   rows 0-31 for A and 32-63 for B, so no phase writes rows another reads.

// BF16 z, SiLU, BF16 h of accumulator block (nt, mt) of half hf (the products started from the
// bias); h into LDS, z (KEEP) to HBM.  Each z is rounded by one conversion, and packed again only
// when it is stored.
template <bool KEEP>
__device__ __attribute__((always_inline)) inline void ws_epi_block(const v4f32& acc, uint16_t* out,
                                                                   uint16_t* __restrict__ zout, int64_t row0,
                                                                   int nvalid, int hf, int nt, int mt, int wv, int g,
                                                                   int r) {
    const int n0 = 32 * wv + 16 * nt + 4 * g;
    const int m = 16 * (2 * hf + mt) + r;
    const uint32_t h01 = f2bf2(silu(bfr(acc[0])), silu(bfr(acc[1])));
    const uint32_t h23 = f2bf2(silu(bfr(acc[2])), silu(bfr(acc[3])));
    *(uint2*)(out + m * LDP + n0) = make_uint2(h01, h23);
    if (KEEP && m < nvalid)
        *(uint2*)(zout + (row0 + m) * HW + n0) = make_uint2(f2bf2(acc[0], acc[1]), f2bf2(acc[2], acc[3]));
}

// accumulators of columns n0 .. n0 + 3 (both sample blocks) set to the bias
__device__ __attribute__((always_inline)) inline void ws_bias(v4f32 (&acc)[2][2], const float* bias, int wv,
                                                              int g) {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const float4 bb = *(const float4*)(bias + 32 * wv + 16 * nt + 4 * g);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) acc[nt][mt] = (v4f32){bb.x, bb.y, bb.z, bb.w};
    }
}

// One phase of a hidden layer: the products of half hm (activations `in`, weights in
// registers, bias `mbias`) into accm, with the epilogue of half he from acce (if EPI)
// spread between them.
template <bool KEEP, bool EPI>
__device__ __attribute__((always_inline)) inline void ws_phase(const uint16_t* in, const v8i16 (&wr)[2][8],
                                                               const float* mbias, int hm, v4f32 (&accm)[2][2],
                                                               const v4f32 (&acce)[2][2], int he, uint16_t* out,
                                                               uint16_t* __restrict__ zout, int64_t row0, int nvalid,
                                                               int wv, int g, int r) {
    v4f32 acc[2][2];
    ws_bias(acc, mbias, wv, g);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        v8i16 b[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) b[mt] = ld8(in + (16 * (2 * hm + mt) + r) * LDP + 32 * ks + 8 * g);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) acc[nt][mt] = mfma32(wr[nt][ks], b[mt], acc[nt][mt]);
        if (EPI && (ks & 1)) {
            const int q = ks >> 1, nt = q >> 1, mt = q & 1;
            ws_epi_block<KEEP>(acce[nt][mt], out, zout, row0, nvalid, he, nt, mt, wv, g, r);
        }
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) accm[nt][mt] = acc[nt][mt];
}

// epilogue of a whole half
template <bool KEEP>
__device__ __attribute__((always_inline)) inline void ws_epi_half(const v4f32 (&acc)[2][2], int hf, uint16_t* out,
                                                                  uint16_t* __restrict__ zout, int64_t row0,
                                                                  int nvalid, int wv, int g, int r) {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) ws_epi_block<KEEP>(acc[nt][mt], out, zout, row0, nvalid, hf, nt, mt, wv, g, r);
}

// layer 1 products of half hf: one k-step of 32 (inputs 16..31 and their weights are zero)
__device__ __attribute__((always_inline)) inline void ws_l1(const uint16_t* sx, const uint16_t* sw1,
                                                            const float* bias, int hf, v4f32 (&acc)[2][2], int wv,
                                                            int g, int r) {
    ws_bias(acc, bias, wv, g);
    v8i16 a[2], b[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) a[nt] = ld8(sw1 + (32 * wv + 16 * nt + r) * LDW1 + 8 * g);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) b[mt] = ld8(sx + (16 * (2 * hf + mt) + r) * LDXP + 8 * g);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) acc[nt][mt] = mfma32(a[nt], b[mt], acc[nt][mt]);
}

template <bool KEEP>
__global__ __launch_bounds__(512, 1) void k_mlp_fwd_ws(const uint16_t* __restrict__ wt, const float* __restrict__ w,
                                                       const uint16_t* __restrict__ X,
                                                       const int32_t* __restrict__ rows, int64_t n,
                                                       float* __restrict__ Y, uint16_t* __restrict__ Z) {
    __shared__ __attribute__((aligned(16))) uint16_t sx[PT * LDXP];
    __shared__ __attribute__((aligned(16))) uint16_t ha[PT * LDP];
    __shared__ __attribute__((aligned(16))) uint16_t hb[PT * LDP];
    __shared__ __attribute__((aligned(16))) uint16_t sw1[HW * LDW1];
    __shared__ __attribute__((aligned(16))) uint16_t sw4[2 * HW];
    __shared__ __attribute__((aligned(16))) float sbias[3 * HW];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int g = lane >> 4, r = lane & 15;
    for (int i = t; i < HW * 32; i += 512) {
        const int nn = i >> 5, k = i & 31;
        sw1[nn * LDW1 + k] = k < DIN ? wt[WT1 + nn * DIN + k] : (uint16_t)0;
    }
    for (int i = t; i < 2 * HW; i += 512) sw4[i] = wt[WT4 + i];
    for (int i = t; i < HW; i += 512) {
        sbias[i] = w[OFF_B1 + i];
        sbias[HW + i] = w[OFF_B2 + i];
        sbias[2 * HW + i] = w[OFF_B3 + i];
    }
    for (int i = t; i < PT * LDXP; i += 512) sx[i] = 0;  // columns 16..31 stay zero
    v8i16 w2r[2][8], w3r[2][8];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const int64_t o = (int64_t)(32 * wv + 16 * nt + r) * HW + 32 * ks + 8 * g;
            w2r[nt][ks] = ld8(wt + WT2 + o);
            w3r[nt][ks] = ld8(wt + WT3 + o);
        }
    const float b40 = w[OFF_B4], b41 = w[OFF_B4 + 1];
    const int64_t tiles = (n + PT - 1) / PT;
    uint16_t* Z1 = KEEP ? Z : nullptr;
    uint16_t* Z2 = KEEP ? Z + n * HW : nullptr;
    uint16_t* Z3 = KEEP ? Z + 2 * n * HW : nullptr;
    // 64 samples x 16 inputs of tile tl into sx, 4 per thread (zero beyond n)
    auto load_x = [&](int64_t tl) {
        if (t < PT * 4) {
            const int64_t r0 = tl * PT;
            const int m = t >> 2, q = t & 3;
            v4i16 v = (v4i16){0, 0, 0, 0};
            if (r0 + m < n) {
                const int64_t src = rows ? (int64_t)rows[r0 + m] : r0 + m;
                v = ld4(X + src * DIN + 4 * q);
            }
            *(v4i16*)(sx + m * LDXP + 4 * q) = v;
        }
    };
    int64_t tile = blockIdx.x;
    if (tile >= tiles) return;  // the grid never exceeds the tile count; every wave leaves together
    load_x(tile);
    __syncthreads();
    v4f32 aA[2][2], aB[2][2];
    ws_l1(sx, sw1, sbias, 0, aA, wv, g, r);
    for (;;) {
        const int64_t row0 = tile * PT;
        const int nvalid = (int)(n - row0 < PT ? n - row0 : PT);
        ws_l1(sx, sw1, sbias, 1, aB, wv, g, r);
        ws_epi_half<KEEP>(aA, 0, ha, Z1, row0, nvalid, wv, g, r);
        __syncthreads();
        ws_phase<KEEP, true>(ha, w2r, sbias + HW, 0, aA, aB, 1, ha, Z1, row0, nvalid, wv, g, r);
        __syncthreads();
        ws_phase<KEEP, true>(ha, w2r, sbias + HW, 1, aB, aA, 0, hb, Z2, row0, nvalid, wv, g, r);
        __syncthreads();
        ws_phase<KEEP, true>(hb, w3r, sbias + 2 * HW, 0, aA, aB, 1, hb, Z2, row0, nvalid, wv, g, r);
        __syncthreads();
        ws_phase<KEEP, true>(hb, w3r, sbias + 2 * HW, 1, aB, aA, 0, ha, Z3, row0, nvalid, wv, g, r);
        __syncthreads();
        ws_epi_half<KEEP>(aB, 1, ha, Z3, row0, nvalid, wv, g, r);
        const int64_t next = tile + gridDim.x;
        if (next < tiles) load_x(next);  // sx was last read by this tile's M(B,1)
        __syncthreads();
        if (wv < 4) {  // head: wave wv takes samples 16 wv .. 16 wv + 15; A = W4t rows 0, 1 (others zero)
            v4f32 acc = (v4f32){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                const v8i16 a = r < 2 ? ld8(sw4 + r * HW + 32 * ks + 8 * g) : (v8i16){0, 0, 0, 0, 0, 0, 0, 0};
                acc = mfma32(a, ld8(ha + (16 * wv + r) * LDP + 32 * ks + 8 * g), acc);
            }
            const int m = 16 * wv + r;
            if (g == 0 && m < nvalid) *(float2*)(Y + (row0 + m) * DOUT) = make_float2(acc[0] + b40, acc[1] + b41);
        }
        if (next >= tiles) break;
        ws_l1(sx, sw1, sbias, 0, aA, wv, g, r);
        __syncthreads();  // the head has read ha before the next tile writes it
        tile = next;
    }
}

// ---------------------------------------------------------------- backward
//
// Three passes.  The signal pass takes tiles of 32 samples through the layers
// in reverse: dZ3 from the head, then dZ2 = bf16((dZ3 W3^T) silu'(z2)) and dZ1
// likewise, the products on v_mfma_f32_16x16x32_bf16 with dZ in LDS (A
// operand, rows = samples) and the BF16 weights in their [K][N] copy read
// from L2 (B operand; wave w owns the 64 columns [64w, 64w+64)).  It writes
// dZ1..dZ3, the activations h1, h2 and the (row-selected) inputs transposed,
// as [feature][sample] arrays over the padded sample range (zero beyond n),
// and accumulates the small gradients (W4, b4, the biases), which are owned
// column by column, in registers over its tiles.  The weight pass forms
// dW = H^T dZ for W1..W3 over chunks of samples: both operands are rows of
// the transposed arrays, so a lane's 8 consecutive samples are one 16-byte
// load straight into registers; a workgroup owns a 64 x 64 block of W2 or W3
// (16 x 64 of W1) and one chunk, its four waves interleave the chunk's
// 32-sample steps and are summed in LDS in wave order.  The last pass adds
// the chunk and workgroup partials, in order, to the gradients, so the
// result is deterministic.
constexpr int BT = 32;  // samples per signal-pass tile
// per-workgroup small partials: W4 [256][2], b4, b3, b2, b1
constexpr int SP_W4 = 0, SP_B4 = SP_W4 + HW * DOUT, SP_B3 = SP_B4 + DOUT, SP_B2 = SP_B3 + HW, SP_B1 = SP_B2 + HW;
constexpr int SMALLP = (SP_B1 + HW + 7) / 8 * 8;
// per-chunk partials: W1 [16][256], W2, W3 [256][256], then the chunk's share of the small partials
constexpr int64_t BP_W1 = 0, BP_W2 = BP_W1 + DIN * HW, BP_W3 = BP_W2 + HW * HW, BP_SMALL = BP_W3 + HW * HW,
                  NBIG = BP_SMALL + SMALLP;
constexpr int SMALL_JOBS = (SMALLP + 255) / 256;  // weight-pass jobs summing the small partials
constexpr int WG_JOBS = 36 + SMALL_JOBS;         // weight-pass jobs per chunk
constexpr int MAX_WCHUNKS = 64;

constexpr int SIG_THREADS = 512;  // signal-pass workgroup: 8 waves; thread (j, hs) owns column j, half hs
constexpr int SIG_HALF = BT / 2;   // samples of a half

// Rows [0, 32) of a Z tile (zero beyond nvalid): the thread's share loaded into registers
// (all three layers' tiles are fetched together at the start of a tile) and later put in LDS.
constexpr int ZPT = BT * HW / 8 / SIG_THREADS;  // 16-byte pieces per thread
__device__ inline void bwd_fetch_z(const uint16_t* __restrict__ Z, uint4 (&v)[ZPT], int64_t row0, int nvalid) {
#pragma unroll
    for (int i = 0; i < ZPT; ++i) {
        const int idx = threadIdx.x + SIG_THREADS * i, m = idx >> 5, c = idx & 31;
        v[i] = m < nvalid ? *(const uint4*)(Z + (row0 + m) * HW + 8 * c) : make_uint4(0, 0, 0, 0);
    }
}
__device__ inline void bwd_put_z(const uint4 (&v)[ZPT], uint16_t* s) {
#pragma unroll
    for (int i = 0; i < ZPT; ++i) {
        const int idx = threadIdx.x + SIG_THREADS * i, m = idx >> 5, c = idx & 31;
        *(uint4*)(s + m * LDH + 8 * c) = v[i];
    }
}

// HT[j][row0 + m] = bf16(silu(z[m][j])) for the thread's column j and half hs (zero beyond nvalid)
__device__ inline void bwd_store_ht(const uint16_t* sz, uint16_t* __restrict__ HT, int64_t npad, int64_t row0,
                                    int nvalid, int j, int hs) {
#pragma unroll
    for (int q = 0; q < SIG_HALF / 8; ++q) {
        uint32_t p[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = SIG_HALF * hs + 8 * q + 2 * i;
            const float h0 = m < nvalid ? silu(bf2f(sz[m * LDH + j])) : 0.f;
            const float h1 = m + 1 < nvalid ? silu(bf2f(sz[(m + 1) * LDH + j])) : 0.f;
            p[i] = f2bf2(h0, h1);
        }
        *(uint4*)(HT + (int64_t)j * npad + row0 + SIG_HALF * hs + 8 * q) = make_uint4(p[0], p[1], p[2], p[3]);
    }
}

// The wave's B operands of a weight matrix for all 8 k-steps (W as the [K][N] copy, rows
// j in [32w, 32w+32)), loaded ahead of the product that uses them.
__device__ __attribute__((always_inline)) inline void bwd_load_w(const uint16_t* __restrict__ Wb,
                                                                 v8i16 (&wf)[8][2]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) wf[ks][nt] = ld8(Wb + (int64_t)(32 * wv + 16 * nt + r) * HW + 32 * ks + 8 * g);
}

// dZ_prev[m][j] = bf16((sum_n dZ[m][n] W[j][n]) silu'(z[m][j])) for the tile: dZ in sd
// (replaced by dZ_prev), z in sz, W's fragments in wf; dZ_prev also to dZT[j][sample].
// Once the products are issued, wf is refilled from Wnext for the next product.
__device__ __attribute__((always_inline)) inline void bwd_signal_layer(uint16_t* sd, const uint16_t* sz,
                                                                       v8i16 (&wf)[8][2],
                                                                       const uint16_t* __restrict__ Wnext,
                                                                       uint16_t* __restrict__ dZT, int64_t npad,
                                                                       int64_t row0, int nvalid) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    v4f32 acc[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = (v4f32){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        v8i16 a[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) a[mt] = ld8(sd + (16 * mt + r) * LDH + 32 * ks + 8 * g);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = mfma32(a[mt], wf[ks][nt], acc[mt][nt]);
    }
    bwd_load_w(Wnext, wf);
    __syncthreads();  // every wave has read dZ before it is replaced
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int j = 32 * wv + 16 * nt + r, m0 = 16 * mt + 4 * g;
            uint16_t d[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + i;
                d[i] = m < nvalid ? f2bf(acc[mt][nt][i] * dsilu(bf2f(sz[m * LDH + j]))) : (uint16_t)0;
                sd[m * LDH + j] = d[i];
            }
            *(uint2*)(dZT + (int64_t)j * npad + row0 + m0) =
                make_uint2((uint32_t)d[0] | ((uint32_t)d[1] << 16), (uint32_t)d[2] | ((uint32_t)d[3] << 16));
        }
}

// Signal pass over tiles blockIdx.x, +gridDim.x, ...; T holds dZT3, dZT2, dZT1, HT2, HT1
// ([256][npad] each), XT the inputs [16][npad]; sp[blockIdx.x][SMALLP] the small partials.
__global__ __launch_bounds__(SIG_THREADS, 1) void k_bwd_signal(const uint16_t* __restrict__ wb,
                                                               const float* __restrict__ w,
                                                               const uint16_t* __restrict__ X,
                                                               const int32_t* __restrict__ rows, int64_t n,
                                                               int64_t npad, const uint16_t* __restrict__ Z,
                                                               const float* __restrict__ dY, uint16_t* __restrict__ T,
                                                               uint16_t* __restrict__ XT, float* __restrict__ sp) {
    __shared__ __attribute__((aligned(16))) uint16_t sd[BT * LDH];  // dZ of the current layer, [m][j]
    __shared__ __attribute__((aligned(16))) uint16_t sz[BT * LDH];  // z of the layer below, [m][j]
    __shared__ float sdy[BT * DOUT];
    __shared__ float sred[6 * HW];  // the second half's column partials, added in a fixed order
    const int t = threadIdx.x, j = t & (HW - 1), hs = t / HW;
    const int64_t tiles = npad / BT, plane = HW * npad;
    const uint16_t* Z1 = Z;
    const uint16_t* Z2 = Z + n * HW;
    const uint16_t* Z3 = Z + 2 * n * HW;
    uint16_t* dZT3 = T;
    uint16_t* dZT2 = T + plane;
    uint16_t* dZT1 = T + 2 * plane;
    uint16_t* HT2 = T + 3 * plane;
    uint16_t* HT1 = T + 4 * plane;
    const float w40 = bf2f(f2bf(w[OFF_W4 + j * DOUT])), w41 = bf2f(f2bf(w[OFF_W4 + j * DOUT + 1]));
    float gw0 = 0.f, gw1 = 0.f, gb3 = 0.f, gb2 = 0.f, gb1 = 0.f, gb4 = 0.f;  // partials of column j, half hs
    v8i16 wf[8][2];
    bwd_load_w(wb + WB3, wf);
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t row0 = tile * BT;
        const int nvalid = (int)(n - row0 < BT ? n - row0 : BT);
        if (t < BT * DOUT) {
            const int m = t / DOUT;
            sdy[t] = m < nvalid ? dY[(row0 + m) * DOUT + (t % DOUT)] : 0.f;
        }
        if (t < DIN * (BT / 8)) {  // inputs, transposed: thread (k, q) writes x[8q .. 8q+7][k]
            const int k = t & (DIN - 1), q = t / DIN;
            uint32_t p[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                uint32_t lo = 0, hi = 0;
                const int m = 8 * q + 2 * i;
                if (m < nvalid) lo = X[(rows ? (int64_t)rows[row0 + m] : row0 + m) * DIN + k];
                if (m + 1 < nvalid) hi = X[(rows ? (int64_t)rows[row0 + m + 1] : row0 + m + 1) * DIN + k];
                p[i] = lo | (hi << 16);
            }
            *(uint4*)(XT + (int64_t)k * npad + row0 + 8 * q) = make_uint4(p[0], p[1], p[2], p[3]);
        }
        uint4 z3[ZPT], z2[ZPT], z1[ZPT];
        bwd_fetch_z(Z3, z3, row0, nvalid);
        bwd_fetch_z(Z2, z2, row0, nvalid);
        bwd_fetch_z(Z1, z1, row0, nvalid);
        bwd_put_z(z3, sz);
        __syncthreads();
        // head, column j, samples of half hs: dW4[j][c] += sum_m h3[m][j] dY[m][c];
        // dZ3 = bf16((dY W4^T) silu'(z3))
        {
#pragma unroll 1
            for (int q = 0; q < SIG_HALF / 8; ++q) {
                uint32_t p[4];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int m = SIG_HALF * hs + 8 * q + i;
                    const float z = bf2f(sz[m * LDH + j]);
                    const bool ok = m < nvalid;
                    const float h = ok ? bf2f(f2bf(silu(z))) : 0.f;
                    const float d0 = sdy[m * DOUT], d1 = sdy[m * DOUT + 1];
                    gw0 += h * d0;
                    gw1 += h * d1;
                    const uint16_t dz = ok ? f2bf((d0 * w40 + d1 * w41) * dsilu(z)) : (uint16_t)0;
                    sd[m * LDH + j] = dz;
                    gb3 += bf2f(dz);
                    if (i & 1) p[i >> 1] |= (uint32_t)dz << 16;
                    else p[i >> 1] = dz;
                }
                *(uint4*)(dZT3 + (int64_t)j * npad + row0 + SIG_HALF * hs + 8 * q) = make_uint4(p[0], p[1], p[2], p[3]);
            }
            if (j < DOUT)
                for (int m = SIG_HALF * hs; m < SIG_HALF * (hs + 1); ++m) gb4 += sdy[m * DOUT + j];
        }
        __syncthreads();  // sz (z3) and sdy are read
        bwd_put_z(z2, sz);
        __syncthreads();
        bwd_store_ht(sz, HT2, npad, row0, nvalid, j, hs);
        bwd_signal_layer(sd, sz, wf, wb + WB2, dZT2, npad, row0, nvalid);
        __syncthreads();
        for (int m = SIG_HALF * hs; m < SIG_HALF * (hs + 1); ++m) gb2 += bf2f(sd[m * LDH + j]);
        bwd_put_z(z1, sz);
        __syncthreads();
        bwd_store_ht(sz, HT1, npad, row0, nvalid, j, hs);
        bwd_signal_layer(sd, sz, wf, wb + WB3, dZT1, npad, row0, nvalid);  // W3 again for the next tile
        __syncthreads();
        for (int m = SIG_HALF * hs; m < SIG_HALF * (hs + 1); ++m) gb1 += bf2f(sd[m * LDH + j]);
        __syncthreads();  // before the next tile overwrites sd, sz, sdy
    }
    if (hs == 1) {
        sred[0 * HW + j] = gw0;
        sred[1 * HW + j] = gw1;
        sred[2 * HW + j] = gb3;
        sred[3 * HW + j] = gb2;
        sred[4 * HW + j] = gb1;
        sred[5 * HW + j] = gb4;
    }
    __syncthreads();
    if (hs == 0) {
        float* part = sp + blockIdx.x * (int64_t)SMALLP;
        part[SP_W4 + j * DOUT] = gw0 + sred[0 * HW + j];
        part[SP_W4 + j * DOUT + 1] = gw1 + sred[1 * HW + j];
        part[SP_B3 + j] = gb3 + sred[2 * HW + j];
        part[SP_B2 + j] = gb2 + sred[3 * HW + j];
        part[SP_B1 + j] = gb1 + sred[4 * HW + j];
        if (j < DOUT) part[SP_B4 + j] = gb4 + sred[5 * HW + j];
    }
}

// One 16*MTA x 64 block of dW = A^T B over the 32-sample steps [s0, s1) of the
// transposed arrays (A rows a0.., B rows b0.., leading dimension npad): wave w
// takes steps s0 + w, s0 + w + 4, ...; the four waves are summed through LDS
// in wave order and the block goes to out[row][col] (row stride ldo).
template <int MTA>
__device__ __attribute__((always_inline)) inline void wgrad_block(const uint16_t* __restrict__ A,
                                                                  const uint16_t* __restrict__ B, int64_t npad,
                                                                  int64_t s0, int64_t s1, float* red,
                                                                  float* __restrict__ out, int ldo) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    v4f32 acc[MTA][4];
#pragma unroll
    for (int mt = 0; mt < MTA; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = (v4f32){0.f, 0.f, 0.f, 0.f};
    const uint16_t* pa = A + (int64_t)r * npad + 8 * g;
    const uint16_t* pb = B + (int64_t)r * npad + 8 * g;
    int64_t s = s0 + wv;
    v8i16 a[MTA], b[4];
    if (s < s1) {  // the next step's operands are loaded while this step's products run
#pragma unroll
        for (int mt = 0; mt < MTA; ++mt) a[mt] = ld8(pa + 16 * mt * npad + 32 * s);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) b[nt] = ld8(pb + 16 * nt * npad + 32 * s);
    }
    for (; s < s1; s += 4) {
        const bool more = s + 4 < s1;
        v8i16 an[MTA], bn[4];
        if (more) {
#pragma unroll
            for (int mt = 0; mt < MTA; ++mt) an[mt] = ld8(pa + 16 * mt * npad + 32 * (s + 4));
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) bn[nt] = ld8(pb + 16 * nt * npad + 32 * (s + 4));
        }
#pragma unroll
        for (int mt = 0; mt < MTA; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mfma32(a[mt], b[nt], acc[mt][nt]);
        if (more) {
#pragma unroll
            for (int mt = 0; mt < MTA; ++mt) a[mt] = an[mt];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) b[nt] = bn[nt];
        }
    }
    constexpr int PER_WAVE = MTA * 4 * 4 * 64;
#pragma unroll
    for (int mt = 0; mt < MTA; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[wv * PER_WAVE + ((mt * 4 + nt) * 4 + i) * 64 + lane] = acc[mt][nt][i];
    __syncthreads();
    for (int e = threadIdx.x; e < PER_WAVE; e += 256) {
        const float v = ((red[e] + red[PER_WAVE + e]) + red[2 * PER_WAVE + e]) + red[3 * PER_WAVE + e];
        const int ln = e & 63, q = e >> 6, i = q & 3, nt = (q >> 2) & 3, mt = q >> 4;
        out[(16 * mt + 4 * (ln >> 4) + i) * ldo + 16 * nt + (ln & 15)] = v;
    }
}

// Weight pass: workgroup b takes chunk b % n_chunks of job b / n_chunks; jobs 0..15 are the
// 64 x 64 blocks of W3 (H2^T dZ3), 16..31 those of W2 (H1^T dZ2), 32..35 the
// 16 x 64 blocks of W1 (X^T dZ1), and jobs 36.. add the chunk's share of the signal pass's
// small partials (its groups, in order; 256 of them per job).  bp[chunk][NBIG] receives the
// chunk's partials.
__global__ __launch_bounds__(256) void k_bwd_wgrad(const uint16_t* __restrict__ T, const uint16_t* __restrict__ XT,
                                                    int64_t npad, int n_chunks, const float* __restrict__ sp,
                                                    int n_groups, float* __restrict__ bp) {
    __shared__ __attribute__((aligned(16))) float red[4 * 4 * 4 * 4 * 64];
    const int64_t plane = HW * npad;
    const int chunk = (int)(blockIdx.x % n_chunks), job = (int)(blockIdx.x / n_chunks);
    const int64_t steps = npad / 32, per = (steps + n_chunks - 1) / n_chunks;
    const int64_t s0 = chunk * per, s1 = s0 + per < steps ? s0 + per : steps;
    float* base = bp + chunk * NBIG;
    if (job >= 36) {
        const int g0 = (int)((int64_t)chunk * n_groups / n_chunks), g1 = (int)((int64_t)(chunk + 1) * n_groups / n_chunks);
        const int i = (job - 36) * 256 + threadIdx.x;
        if (i < SMALLP) {
            float acc = 0.f;
#pragma unroll 8
            for (int gi = g0; gi < g1; ++gi) acc += sp[(int64_t)gi * SMALLP + i];
            base[BP_SMALL + i] = acc;
        }
        return;
    }
    if (job < 32) {
        const int mat = job < 16 ? 3 : 2, blk = job & 15, jb = blk >> 2, nb4 = blk & 3;
        const uint16_t* A = (mat == 3 ? T + 3 * plane : T + 4 * plane) + (int64_t)(64 * jb) * npad;  // HT2 / HT1
        const uint16_t* B = (mat == 3 ? T : T + plane) + (int64_t)(64 * nb4) * npad;                // dZT3 / dZT2
        float* out = base + (mat == 3 ? BP_W3 : BP_W2) + (64 * jb) * HW + 64 * nb4;
        wgrad_block<4>(A, B, npad, s0, s1, red, out, HW);
    } else {
        const int nb4 = job - 32;
        wgrad_block<1>(XT, T + 2 * plane + (int64_t)(64 * nb4) * npad, npad, s0, s1, red, base + BP_W1 + 64 * nb4,
                       HW);
    }
}

// grad[p] += the chunk partials of p, in chunk order
__global__ void k_grad_sum(const float* __restrict__ bp, int n_chunks, float* __restrict__ grad) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    int64_t src;
    if (p < OFF_B1) src = BP_W1 + (p - OFF_W1);
    else if (p < OFF_W2) src = BP_SMALL + SP_B1 + (p - OFF_B1);
    else if (p < OFF_B2) src = BP_W2 + (p - OFF_W2);
    else if (p < OFF_W3) src = BP_SMALL + SP_B2 + (p - OFF_B2);
    else if (p < OFF_B3) src = BP_W3 + (p - OFF_W3);
    else if (p < OFF_W4) src = BP_SMALL + SP_B3 + (p - OFF_B3);
    else if (p < OFF_B4) src = BP_SMALL + SP_W4 + (p - OFF_W4);
    else src = BP_SMALL + SP_B4 + (p - OFF_B4);
    float s = 0.f;
    for (int c = 0; c < n_chunks; ++c) s += bp[(int64_t)c * NBIG + src];
    grad[p] += s;
}

// mean Gaussian NLL: 0.5 (exp(-s) (t - m)^2 + s); dY for the mean over n samples
__global__ void k_nll(const float* __restrict__ Y, const float* __restrict__ T, const int32_t* __restrict__ rows,
                      int64_t n, float* __restrict__ dY, float* __restrict__ loss_sum) {
    __shared__ float red[256];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    float l = 0.f;
    if (i < n) {
        const float m = Y[2 * i], s = Y[2 * i + 1];
        const float t = T[rows ? (int64_t)rows[i] : i];
        const float e = __expf(-s), d = t - m;
        l = 0.5f * (e * d * d + s);
        dY[2 * i] = -(e * d) / (float)n;
        dY[2 * i + 1] = 0.5f * (1.f - e * d * d) / (float)n;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss_sum) atomicAdd(loss_sum, red[0]);
}

__device__ inline void adam_one(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, int64_t i, float lr, float b1, float b2, float eps, float wd,
                                float c1, float c2) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * w[i]);
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float wd, float c1, float c2) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    adam_one(w, g, m, v, i, lr, b1, b2, eps, wd, c1, c2);
}

// bias correction 1 - b^t, formed in FP64 and rounded once (host and device agree)
__host__ __device__ inline float bias_corr(float b, int64_t t) { return (float)(1.0 - pow((double)b, (double)t)); }

// ---------------------------------------------------------------- training steps on the device
//
// The step number k lives in device memory, so one captured step serves every
// replay: rows drawn from (seed, k), the cosine learning rate of k, the bias
// corrections of k + 1, then k += 1.
__global__ void k_set_step(int64_t* __restrict__ st, int64_t v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *st = v;
}

__global__ void k_step_inc(int64_t* __restrict__ st) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *st += 1;
}

__global__ void k_train_rows(const int64_t* __restrict__ st, uint64_t seed, int64_t N, int64_t batch,
                             int32_t* __restrict__ rows) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= batch) return;
    const uint64_t k = (uint64_t)*st;
    uint64_t z = seed + (k * (uint64_t)batch + (uint64_t)i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    rows[i] = (int32_t)(z % (uint64_t)N);
}

__global__ void k_zero_f32(float* __restrict__ p, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

__global__ void k_adam_sched(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                             float* __restrict__ v, const int64_t* __restrict__ st, rt_train_opts o) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    const int64_t k = *st;
    const double frac = (double)(k < o.total_steps ? k : o.total_steps) / (double)o.total_steps;
    const float lr = (float)((double)o.lr_final +
                             0.5 * ((double)o.lr - (double)o.lr_final) * (1.0 + cos(3.141592653589793 * frac)));
    adam_one(w, g, m, v, i, lr, o.b1, o.b2, o.eps, o.wd, bias_corr(o.b1, k + 1), bias_corr(o.b2, k + 1));
}

// ---------------------------------------------------------------- features

// feat[(k*F + f)*16 + c] for point p = points[k] (or p = k) at frequency f;
// J1 is [n_points][F] in the same order.  Features (c): 0 log J1, 1 log chi,
// 2 log S, 3/4 neighbour mean of log chi / log S, 5 neighbour standard
// deviation of log chi, 6/7 the eq. 6 indicator max_n |(f_p - f_n)/(f_p + f_n)|
// of chi and S, 8 log L_p with L_p the mean neighbour distance (eq. 8),
// 9 log(chi L_p), 10 x_f / 5, 11 log(number of neighbours); 12, 13, 14 the
// max, min and standard deviation over the R coarse pairs of log(u_r / J1)
// when u [n_points][R][F] is given (else zero); 15 zero.
__global__ void k_features(const double* __restrict__ pos, const int64_t* __restrict__ off,
                           const int32_t* __restrict__ idx, const float* __restrict__ chi,
                           const float* __restrict__ eta, int64_t ld, int64_t F, const float* __restrict__ fx,
                           const float* __restrict__ J1, const float* __restrict__ u, int64_t R,
                           const int32_t* __restrict__ points, int64_t n_points, int64_t P,
                           float* __restrict__ feat, int32_t* __restrict__ err) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_points * F) return;
    const int64_t k = i / F;
    const int64_t f = i - k * F;
    const int64_t p = points ? (int64_t)points[k] : k;
    if (p < 0 || p >= P) {
        if (err) atomicOr(err, ERRBIT_ORIGIN);
        for (int c = 0; c < DIN; ++c) feat[i * DIN + c] = 0.f;
        return;
    }
    const float cp = chi[p * ld + f], sp = eta[p * ld + f] / cp;
    const int64_t e0 = off[p], e1 = off[p + 1];
    const double px = pos[3 * p], py = pos[3 * p + 1], pz = pos[3 * p + 2];
    float s_lc = 0.f, s_ls = 0.f, gc = 0.f, gs = 0.f;
    double L = 0.0;
    for (int64_t e = e0; e < e1; ++e) {
        const int64_t q = idx[e];
        const float cq = chi[q * ld + f], sq = eta[q * ld + f] / cq;
        s_lc += logf(cq);
        s_ls += logf(sq);
        gc = fmaxf(gc, fabsf((cp - cq) / (cp + cq)));
        gs = fmaxf(gs, fabsf((sp - sq) / (sp + sq)));
        const double dx = pos[3 * q] - px, dy = pos[3 * q + 1] - py, dz = pos[3 * q + 2] - pz;
        L += sqrt(dx * dx + dy * dy + dz * dz);
    }
    const float nd = (float)(e1 - e0);
    const float mlc = s_lc / nd;
    float var = 0.f;
    for (int64_t e = e0; e < e1; ++e) {
        const float d = logf(chi[(int64_t)idx[e] * ld + f]) - mlc;
        var += d * d;
    }
    const float Lp = (float)(L / (double)(e1 - e0));
    float* o = feat + i * DIN;
    o[0] = logf(J1[k * F + f]);
    o[1] = logf(cp);
    o[2] = logf(sp);
    o[3] = mlc;
    o[4] = s_ls / nd;
    o[5] = sqrtf(var / nd);
    o[6] = gc;
    o[7] = gs;
    o[8] = logf(Lp);
    o[9] = logf(cp * Lp);
    o[10] = fx[f] / 5.f;
    o[11] = logf(nd);
    float amax = 0.f, amin = 0.f, asd = 0.f;
    if (u) {
        const float lj = logf(J1[k * F + f]);
        float s1 = 0.f;
        amax = -INFINITY;
        amin = INFINITY;
        for (int64_t r = 0; r < R; ++r) {
            const float a = logf(fmaxf(u[(k * R + r) * F + f], 1e-30f)) - lj;
            amax = fmaxf(amax, a);
            amin = fminf(amin, a);
            s1 += a;
        }
        const float ma = s1 / (float)R;
        for (int64_t r = 0; r < R; ++r) {
            const float d = logf(fmaxf(u[(k * R + r) * F + f], 1e-30f)) - lj - ma;
            asd += d * d;
        }
        asd = sqrtf(asd / (float)R);
    }
    o[12] = amax;
    o[13] = amin;
    o[14] = asd;
    o[15] = 0.f;
}

// Column sums and sums of squares of feat[n][16]: block b accumulates rows
// b*256 + t + k*STAT_BLOCKS*256 per thread, reduces in a fixed order and
// writes part[b][32]; k_feature_stats_final sums the blocks in order.
constexpr int STAT_BLOCKS = RT_CLOSURE_STAT_BLOCKS;

__global__ __launch_bounds__(256) void k_feature_stats(const float* __restrict__ feat, int64_t n,
                                                        double* __restrict__ part) {
    __shared__ double sw[4][2 * DIN];
    double acc[2 * DIN];
#pragma unroll
    for (int c = 0; c < 2 * DIN; ++c) acc[c] = 0.0;
    for (int64_t r = blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)STAT_BLOCKS * 256) {
#pragma unroll
        for (int c = 0; c < DIN; ++c) {
            const double v = feat[r * DIN + c];
            acc[c] += v;
            acc[DIN + c] += v * v;
        }
    }
#pragma unroll
    for (int c = 0; c < 2 * DIN; ++c)
        for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 2 * DIN; ++c) sw[w][c] = acc[c];
    __syncthreads();
    if (threadIdx.x < 2 * DIN)
        part[blockIdx.x * 2 * DIN + threadIdx.x] =
            ((sw[0][threadIdx.x] + sw[1][threadIdx.x]) + sw[2][threadIdx.x]) + sw[3][threadIdx.x];
}

__global__ void k_feature_stats_final(const double* __restrict__ part, double* __restrict__ sums) {
    const int c = threadIdx.x;
    if (c >= 2 * DIN) return;
    double s = 0.0;
    for (int b = 0; b < STAT_BLOCKS; ++b) s += part[b * 2 * DIN + c];
    sums[c] = s;
}

struct Norm {
    float mean[DIN], istd[DIN];
};

__global__ void k_normalize(const float* __restrict__ feat, int64_t n, const Norm nm, uint16_t* __restrict__ X) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * DIN;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % DIN);
        X[i] = f2bf((feat[i] - nm.mean[c]) * nm.istd[c]);
    }
}

// ---------------------------------------------------------------- closure assembly

// Points p0 .. p0+n_points-1 (J1, Y and J start at point p0).
__global__ void k_closure_apply(const float* __restrict__ J1, const float* __restrict__ Y, int64_t n_points,
                                int64_t F, float log_bound, float* __restrict__ J, int32_t* __restrict__ flagged,
                                int32_t* __restrict__ n_flagged, int64_t p0) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n_points) return;
    bool fl = false;
    for (int64_t f = 0; f < F; ++f) {
        const int64_t i = p * F + f;
        J[i] = J1[i] * __expf(Y[2 * i]);
        fl = fl || (0.5f * Y[2 * i + 1] > log_bound);
    }
    if (fl) flagged[atomicAdd(n_flagged, 1)] = (int32_t)(p0 + p);
}

__global__ void k_closure_merge(const float* __restrict__ Jf, const int32_t* __restrict__ flagged, int64_t n_flagged,
                                int64_t F, int64_t n_points, float* __restrict__ J, int32_t* __restrict__ err) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_flagged * F;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = i / F, f = i - k * F;
        const int64_t p = flagged[k];
        if (p < 0 || p >= n_points) {
            if (err) atomicOr(err, ERRBIT_ORIGIN);
            continue;
        }
        J[p * F + f] = Jf[i];
    }
}

__global__ void k_targets(const float* __restrict__ J1, const float* __restrict__ Jf, int64_t n,
                          float* __restrict__ T) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        T[i] = logf(Jf[i] / J1[i]);
}

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

}  // namespace rt

using namespace rt;

struct rt_mlp {
    float* w = nullptr;     // master parameters
    float* g = nullptr;     // gradients
    float* m = nullptr;     // Adam moments
    float* v = nullptr;
    uint16_t* wt = nullptr; // BF16 forward copies
    uint16_t* wb = nullptr; // BF16 backward copies
    int64_t step = 0;
    bool has_norm = false;  // input standardisation for rt_closure_J
    float mean[DIN] = {}, istd[DIN] = {};
    // the captured training step of the last rt_mlp_train call and what it was captured for
    hipGraph_t train_graph = nullptr;
    hipGraphExec_t train_exec = nullptr;
    const void* train_key[5] = {};
    int64_t train_N = 0;
    size_t train_ws_bytes = 0;
    rt_train_opts train_opts = {};
};

static rt_status mlp_publish(rt_mlp* h, hipStream_t s) {
    hipLaunchKernelGGL(k_publish, dim3(nb(HW * HW, 256)), dim3(256), 0, s, h->w, h->wt, h->wb);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status rt_mlp_num_params(int64_t* n) {
    if (!n) return fail(RT_ERR_ARG, "rt_mlp_num_params: NULL");
    *n = NPARAM;
    return RT_OK;
}

extern "C" rt_status rt_mlp_create(uint64_t seed, void* stream, rt_mlp** out) {
    if (!out) return fail(RT_ERR_ARG, "rt_mlp_create: NULL output");
    *out = nullptr;
    auto* h = new rt_mlp();
    hipError_t e = hipMalloc((void**)&h->w, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc((void**)&h->g, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc((void**)&h->m, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc((void**)&h->v, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc((void**)&h->wt, sizeof(uint16_t) * NWT);
    if (e == hipSuccess) e = hipMalloc((void**)&h->wb, sizeof(uint16_t) * NWB);
    // He-style initialisation: weights N(0, 2/fan_in) for the SiLU layers, N(0, 1/fan_in) for the head; biases 0
    std::vector<float> p((size_t)NPARAM, 0.f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.f, 1.f);
    auto fill = [&](int64_t ofs, int64_t cnt, float sd) {
        for (int64_t i = 0; i < cnt; ++i) p[(size_t)(ofs + i)] = sd * nd(rng);
    };
    fill(OFF_W1, DIN * HW, std::sqrt(2.f / 12.f));
    fill(OFF_W2, HW * HW, std::sqrt(2.f / HW));
    fill(OFF_W3, HW * HW, std::sqrt(2.f / HW));
    fill(OFF_W4, HW * DOUT, std::sqrt(1.f / HW));
    hipStream_t s = (hipStream_t)stream;
    if (e == hipSuccess) e = hipMemcpyAsync(h->w, p.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(h->g, 0, sizeof(float) * NPARAM, s);
    if (e == hipSuccess) e = hipMemsetAsync(h->m, 0, sizeof(float) * NPARAM, s);
    if (e == hipSuccess) e = hipMemsetAsync(h->v, 0, sizeof(float) * NPARAM, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        rt_status st = hip_fail(e, "rt_mlp_create");
        rt_mlp_destroy(h);
        return st;
    }
    rt_status st = mlp_publish(h, s);
    if (st) {
        rt_mlp_destroy(h);
        return st;
    }
    *out = h;
    return RT_OK;
}

extern "C" rt_status rt_mlp_destroy(rt_mlp* h) {
    if (!h) return RT_OK;
    if (h->train_exec) (void)hipGraphExecDestroy(h->train_exec);
    if (h->train_graph) (void)hipGraphDestroy(h->train_graph);
    for (void* q : {(void*)h->w, (void*)h->g, (void*)h->m, (void*)h->v, (void*)h->wt, (void*)h->wb})
        if (q) (void)hipFree(q);
    delete h;
    return RT_OK;
}

extern "C" rt_status rt_mlp_get_params(const rt_mlp* h, float* host, void* stream) {
    if (!h || !host) return fail(RT_ERR_ARG, "rt_mlp_get_params: NULL");
    RT_HIP(hipMemcpyAsync(host, h->w, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, (hipStream_t)stream));
    RT_HIP(hipStreamSynchronize((hipStream_t)stream));
    return RT_OK;
}

extern "C" rt_status rt_mlp_set_params(rt_mlp* h, const float* host, void* stream) {
    if (!h || !host) return fail(RT_ERR_ARG, "rt_mlp_set_params: NULL");
    hipStream_t s = (hipStream_t)stream;
    RT_HIP(hipMemcpyAsync(h->w, host, sizeof(float) * NPARAM, hipMemcpyHostToDevice, s));
    RT_HIP(hipStreamSynchronize(s));
    return mlp_publish(h, s);
}

extern "C" rt_status rt_mlp_get_grads(const rt_mlp* h, float* host, void* stream) {
    if (!h || !host) return fail(RT_ERR_ARG, "rt_mlp_get_grads: NULL");
    RT_HIP(hipMemcpyAsync(host, h->g, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, (hipStream_t)stream));
    RT_HIP(hipStreamSynchronize((hipStream_t)stream));
    return RT_OK;
}

extern "C" rt_status rt_mlp_zero_grad(rt_mlp* h, void* stream) {
    if (!h) return fail(RT_ERR_ARG, "rt_mlp_zero_grad: NULL");
    RT_HIP(hipMemsetAsync(h->g, 0, sizeof(float) * NPARAM, (hipStream_t)stream));
    return RT_OK;
}

// Training workspace (each part 256-byte aligned): the BF16 pre-activations
// Z[3][n][256] that the forward keeps; the backward's transposed arrays
// dZ3, dZ2, dZ1, h2, h1 [256][npad] and x [16][npad] (BF16, npad = n rounded
// up to 32); the signal pass's small partials [groups][SMALLP] and the weight
// pass's partials [chunks][NBIG] (FP32).
namespace {
struct BwdParts {
    int64_t npad, groups, chunks;
    size_t t, xt, sp, bp, total;
};
inline size_t al256(size_t v) { return (v + 255) / 256 * 256; }
BwdParts bwd_parts(int64_t n) {
    BwdParts b;
    b.npad = (n + BT - 1) / BT * BT;
    b.groups = std::max<int64_t>(1, std::min<int64_t>(b.npad / BT, 4 * (int64_t)num_cus()));
    b.chunks = std::max<int64_t>(1, std::min<int64_t>(b.npad / 32 / 32, MAX_WCHUNKS));
    b.t = al256((size_t)(3 * n * HW) * sizeof(uint16_t));
    b.xt = b.t + al256((size_t)(5 * HW * b.npad) * sizeof(uint16_t));
    b.sp = b.xt + al256((size_t)(DIN * b.npad) * sizeof(uint16_t));
    b.bp = b.sp + al256((size_t)(b.groups * SMALLP) * sizeof(float));
    b.total = b.bp + (size_t)(b.chunks * NBIG) * sizeof(float);
    return b;
}
}  // namespace
static size_t ws_bytes_for(int64_t n) { return bwd_parts(n).total; }

extern "C" rt_status rt_mlp_workspace(int64_t n, int32_t training, size_t* bytes) {
    if (!bytes || n < 0) return fail(RT_ERR_ARG, "rt_mlp_workspace: bad arguments");
    *bytes = training ? ws_bytes_for(n) : 0;
    return RT_OK;
}

extern "C" rt_status rt_mlp_forward(rt_mlp* h, const uint16_t* X, const int32_t* rows, int64_t n, float* Y,
                                    int32_t keep, void* ws, size_t ws_bytes, void* stream) {
    if (!h || (n > 0 && (!X || !Y)) || n < 0 || n > MAX_SAMPLES)
        return fail(RT_ERR_ARG, "rt_mlp_forward: bad arguments");
    if (n == 0) return RT_OK;
    if (keep && (!ws || ws_bytes < ws_bytes_for(n))) return fail(RT_ERR_CAPACITY, "rt_mlp_forward: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    if (n >= WS_MIN_SAMPLES) {  // many samples: persistent workgroups with the weights in registers
        const int64_t tiles = (n + PT - 1) / PT;
        const unsigned grid = (unsigned)std::min<int64_t>(tiles, num_cus());
        if (keep)
            hipLaunchKernelGGL(k_mlp_fwd_ws<true>, dim3(grid), dim3(64 * PWAVES), 0, s, h->wt, h->w, X, rows, n, Y,
                               (uint16_t*)ws);
        else
            hipLaunchKernelGGL(k_mlp_fwd_ws<false>, dim3(grid), dim3(64 * PWAVES), 0, s, h->wt, h->w, X, rows, n, Y,
                               nullptr);
        RT_HIP(hipGetLastError());
        return RT_OK;
    }
    // small batches (training) in 64-sample tiles to fill the chip, large ones in 128
    if (n < (int64_t)num_cus() * 256) {
        if (keep)
            hipLaunchKernelGGL((k_mlp_fwd<true, 4>), dim3(nb(n, 64)), dim3(256), 0, s, h->wt, h->w, X, rows, n, Y,
                               (uint16_t*)ws);
        else
            hipLaunchKernelGGL((k_mlp_fwd<false, 4>), dim3(nb(n, 64)), dim3(256), 0, s, h->wt, h->w, X, rows, n, Y,
                               nullptr);
    } else {
        if (keep)
            hipLaunchKernelGGL((k_mlp_fwd<true, 8>), dim3(nb(n, 128)), dim3(256), 0, s, h->wt, h->w, X, rows, n, Y,
                               (uint16_t*)ws);
        else
            hipLaunchKernelGGL((k_mlp_fwd<false, 8>), dim3(nb(n, 128)), dim3(256), 0, s, h->wt, h->w, X, rows, n, Y,
                               nullptr);
    }
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status rt_mlp_backward(rt_mlp* h, const uint16_t* X, const int32_t* rows, int64_t n, const float* dY,
                                     void* ws, size_t ws_bytes, void* stream) {
    if (!h || (n > 0 && (!X || !dY)) || n < 0 || n > MAX_SAMPLES)
        return fail(RT_ERR_ARG, "rt_mlp_backward: bad arguments");
    if (n == 0) return RT_OK;
    if (!ws || ws_bytes < ws_bytes_for(n)) return fail(RT_ERR_CAPACITY, "rt_mlp_backward: workspace too small");
    const BwdParts b = bwd_parts(n);
    char* base = (char*)ws;
    uint16_t* T = (uint16_t*)(base + b.t);
    uint16_t* XT = (uint16_t*)(base + b.xt);
    float* sp = (float*)(base + b.sp);
    float* bp = (float*)(base + b.bp);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_bwd_signal, dim3((unsigned)b.groups), dim3(SIG_THREADS), 0, s, h->wb, h->w, X, rows, n, b.npad,
                       (const uint16_t*)ws, dY, T, XT, sp);
    hipLaunchKernelGGL(k_bwd_wgrad, dim3((unsigned)(WG_JOBS * b.chunks)), dim3(256), 0, s, T, XT, b.npad,
                       (int)b.chunks, sp, (int)b.groups, bp);
    hipLaunchKernelGGL(k_grad_sum, dim3(nb(NPARAM, 256)), dim3(256), 0, s, bp, (int)b.chunks, h->g);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status rt_mlp_nll(const float* Y, const float* T, const int32_t* rows, int64_t n, float* dY,
                                float* loss_sum, void* stream) {
    if ((n > 0 && (!Y || !T || !dY)) || n < 0 || n > MAX_SAMPLES) return fail(RT_ERR_ARG, "rt_mlp_nll: bad arguments");
    if (n == 0) return RT_OK;
    hipLaunchKernelGGL(k_nll, dim3(nb(n, 256)), dim3(256), 0, (hipStream_t)stream, Y, T, rows, n, dY, loss_sum);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status rt_mlp_adam_step(rt_mlp* h, float lr, float b1, float b2, float eps, float wd, void* stream) {
    if (!h) return fail(RT_ERR_ARG, "rt_mlp_adam_step: NULL");
    h->step += 1;
    const float c1 = bias_corr(b1, h->step), c2 = bias_corr(b2, h->step);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_adam, dim3(nb(NPARAM, 256)), dim3(256), 0, s, h->w, h->g, h->m, h->v, lr, b1, b2, eps, wd,
                       c1, c2);
    RT_HIP(hipGetLastError());
    return mlp_publish(h, s);
}

// Training workspace: batch rows (int32), Y and dY (f32 [batch][2]), the step
// counter, then the forward/backward workspace of the batch.
namespace {
struct TrainParts {
    size_t rows, Y, dY, st, mlp, total;
};
TrainParts train_parts(int64_t batch) {
    TrainParts t;
    t.rows = 0;
    t.Y = t.rows + al256(sizeof(int32_t) * (size_t)batch);
    t.dY = t.Y + al256(sizeof(float) * DOUT * (size_t)batch);
    t.st = t.dY + al256(sizeof(float) * DOUT * (size_t)batch);
    t.mlp = t.st + 256;
    t.total = t.mlp + ws_bytes_for(batch);
    return t;
}

bool same_opts(const rt_train_opts& a, const rt_train_opts& b) {
    return a.batch == b.batch && a.total_steps == b.total_steps && a.lr == b.lr && a.lr_final == b.lr_final &&
           a.b1 == b.b1 && a.b2 == b.b2 && a.eps == b.eps && a.wd == b.wd && a.seed == b.seed;
}

// one training step on stream s (captured by rt_mlp_train)
rt_status train_enqueue(rt_mlp* h, const uint16_t* X, const float* T, int64_t N, const rt_train_opts& o,
                        float* loss_sum, char* ws, hipStream_t s) {
    const TrainParts tp = train_parts(o.batch);
    int32_t* rows = (int32_t*)(ws + tp.rows);
    float* Y = (float*)(ws + tp.Y);
    float* dY = (float*)(ws + tp.dY);
    int64_t* st = (int64_t*)(ws + tp.st);
    void* mws = ws + tp.mlp;
    const size_t mbytes = ws_bytes_for(o.batch);
    hipLaunchKernelGGL(k_train_rows, dim3(nb(o.batch, 256)), dim3(256), 0, s, st, o.seed, N, o.batch, rows);
    RT_HIP(hipGetLastError());
    rt_status e = rt_mlp_forward(h, X, rows, o.batch, Y, 1, mws, mbytes, s);
    if (!e) e = rt_mlp_nll(Y, T, rows, o.batch, dY, loss_sum, s);
    if (e) return e;
    hipLaunchKernelGGL(k_zero_f32, dim3(nb(NPARAM, 256)), dim3(256), 0, s, h->g, NPARAM);
    e = rt_mlp_backward(h, X, rows, o.batch, dY, mws, mbytes, s);
    if (e) return e;
    hipLaunchKernelGGL(k_adam_sched, dim3(nb(NPARAM, 256)), dim3(256), 0, s, h->w, h->g, h->m, h->v, st, o);
    RT_HIP(hipGetLastError());
    e = mlp_publish(h, s);
    if (e) return e;
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, s, st);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
}  // namespace

extern "C" rt_status rt_mlp_train_workspace(int64_t batch, size_t* bytes) {
    if (!bytes || batch < 1 || batch > MAX_SAMPLES) return fail(RT_ERR_ARG, "rt_mlp_train_workspace: bad arguments");
    *bytes = train_parts(batch).total;
    return RT_OK;
}

extern "C" rt_status rt_mlp_train(rt_mlp* h, const uint16_t* X, const float* T, int64_t N, const rt_train_opts* opts,
                                  int64_t n_steps, float* loss_sum, void* ws, size_t ws_bytes, void* stream) {
    if (!h || !X || !T || !opts || !ws || N < 1 || N > MAX_SAMPLES || n_steps < 0)
        return fail(RT_ERR_ARG, "rt_mlp_train: bad arguments");
    const rt_train_opts o = *opts;
    if (o.batch < 1 || o.batch > MAX_SAMPLES || o.total_steps < 1)
        return fail(RT_ERR_ARG, "rt_mlp_train: bad batch or schedule");
    if (ws_bytes < train_parts(o.batch).total) return fail(RT_ERR_CAPACITY, "rt_mlp_train: workspace too small");
    if (n_steps == 0) return RT_OK;
    hipStream_t s = (hipStream_t)stream;
    const void* key[5] = {X, T, loss_sum, ws, nullptr};
    bool reuse = h->train_exec && h->train_N == N && h->train_ws_bytes == ws_bytes && same_opts(h->train_opts, o);
    for (int i = 0; i < 5 && reuse; ++i) reuse = h->train_key[i] == key[i];
    if (!reuse) {
        if (h->train_exec) (void)hipGraphExecDestroy(h->train_exec);
        if (h->train_graph) (void)hipGraphDestroy(h->train_graph);
        h->train_exec = nullptr;
        h->train_graph = nullptr;
        hipStream_t cap = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        rt_status st = RT_OK;
        if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            st = train_enqueue(h, X, T, N, o, loss_sum, (char*)ws, cap);
            e = hipStreamEndCapture(cap, &h->train_graph);
        }
        if (e == hipSuccess && !st) e = hipGraphInstantiate(&h->train_exec, h->train_graph, nullptr, nullptr, 0);
        if (cap) (void)hipStreamDestroy(cap);
        if (st) return st;
        if (e != hipSuccess) return hip_fail(e, "rt_mlp_train: graph capture");
        for (int i = 0; i < 5; ++i) h->train_key[i] = key[i];
        h->train_N = N;
        h->train_ws_bytes = ws_bytes;
        h->train_opts = o;
    }
    int64_t* st = (int64_t*)((char*)ws + train_parts(o.batch).st);
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, st, h->step);
    RT_HIP(hipGetLastError());
    for (int64_t i = 0; i < n_steps; ++i) RT_HIP(hipGraphLaunch(h->train_exec, s));
    h->step += n_steps;
    return RT_OK;
}

extern "C" rt_status rt_closure_features(const rt_model* m, const float* chi, const float* eta, int64_t ld, int64_t F,
                                         const float* freq_x, const float* J1, const float* u, int64_t R,
                                         const int32_t* points, int64_t n_points, float* feat, void* stream) {
    if (!m || !chi || !eta || !freq_x || !J1 || (n_points > 0 && !feat) || F <= 0 || ld < F || n_points < 0 ||
        n_points * F > MAX_SAMPLES || (!points && n_points > m->P) || (u && R <= 0))
        return fail(RT_ERR_ARG, "rt_closure_features: bad arguments");
    if (n_points == 0) return RT_OK;
    hipLaunchKernelGGL(k_features, dim3(nb(n_points * F, 256)), dim3(256), 0, (hipStream_t)stream, m->pos, m->off,
                       m->idx, chi, eta, ld, F, freq_x, J1, u, R, points, n_points, m->P, feat, error_word());
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status rt_closure_feature_stats(const float* feat, int64_t n, double* sums, double* partial,
                                              void* stream) {
    if (!sums || !partial || (n > 0 && !feat) || n < 0)
        return fail(RT_ERR_ARG, "rt_closure_feature_stats: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_feature_stats, dim3(STAT_BLOCKS), dim3(256), 0, s, feat, n, partial);
    hipLaunchKernelGGL(k_feature_stats_final, dim3(1), dim3(64), 0, s, partial, sums);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status rt_closure_normalize(const float* feat, int64_t n, const float* mean, const float* inv_std,
                                          uint16_t* X, void* stream) {
    if (!mean || !inv_std || (n > 0 && (!feat || !X)) || n < 0)
        return fail(RT_ERR_ARG, "rt_closure_normalize: bad arguments");
    if (n == 0) return RT_OK;
    Norm nm;
    std::memcpy(nm.mean, mean, sizeof(nm.mean));
    std::memcpy(nm.istd, inv_std, sizeof(nm.istd));
    hipLaunchKernelGGL(k_normalize, dim3(capped_blocks(nb(n * DIN, 256))), dim3(256), 0, (hipStream_t)stream, feat, n, nm, X);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status rt_closure_apply(const float* J1, const float* Y, int64_t n_points, int64_t F, float log_bound,
                                      float* J, int32_t* flagged, int32_t* n_flagged, void* stream) {
    if ((n_points > 0 && (!J1 || !Y || !J || !flagged)) || !n_flagged || F <= 0 || n_points < 0)
        return fail(RT_ERR_ARG, "rt_closure_apply: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    RT_HIP(launch_fill_i32(n_flagged, 1, 0, s));
    if (n_points == 0) return RT_OK;
    hipLaunchKernelGGL(k_closure_apply, dim3(nb(n_points, 256)), dim3(256), 0, s, J1, Y,
                       n_points, F, log_bound, J, flagged, n_flagged, (int64_t)0);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status rt_closure_merge(const float* J_fine, const int32_t* flagged, int64_t n_flagged, int64_t F,
                                      int64_t n_points, float* J, void* stream) {
    if ((n_flagged > 0 && (!J_fine || !flagged || !J)) || F <= 0 || n_flagged < 0)
        return fail(RT_ERR_ARG, "rt_closure_merge: bad arguments");
    if (n_flagged == 0) return RT_OK;
    hipLaunchKernelGGL(k_closure_merge, dim3(capped_blocks(nb(n_flagged * F, 256))), dim3(256), 0, (hipStream_t)stream, J_fine,
                       flagged, n_flagged, F, n_points, J, error_word());
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status rt_closure_targets(const float* J1, const float* J_fine, int64_t n, float* T, void* stream) {
    if ((n > 0 && (!J1 || !J_fine || !T)) || n < 0) return fail(RT_ERR_ARG, "rt_closure_targets: bad arguments");
    if (n == 0) return RT_OK;
    hipLaunchKernelGGL(k_targets, dim3(capped_blocks(nb(n, 256))), dim3(256), 0, (hipStream_t)stream, J1, J_fine, n, T);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" rt_status rt_mlp_set_input_norm(rt_mlp* h, const float* mean, const float* inv_std) {
    if (!h || !mean || !inv_std) return fail(RT_ERR_ARG, "rt_mlp_set_input_norm: NULL");
    std::memcpy(h->mean, mean, sizeof(h->mean));
    std::memcpy(h->istd, inv_std, sizeof(h->istd));
    h->has_norm = true;
    return RT_OK;
}

// ---------------------------------------------------------------- the closure in one call

namespace {
constexpr int64_t CLOSURE_CHUNK = 65536;  // points per inference chunk

struct ClosureParts {
    size_t J1, u1, x, pts, cnt, feat, X, Y, Jf, total;
};

ClosureParts closure_parts(int64_t P, int64_t R1, int64_t F) {
    ClosureParts c;
    const int64_t pc = std::min<int64_t>(P, CLOSURE_CHUNK);
    c.J1 = 0;
    c.u1 = c.J1 + al256(sizeof(float) * (size_t)(P * F));
    c.x = c.u1 + al256(sizeof(float) * (size_t)(P * R1 * F));
    c.pts = c.x + al256(sizeof(float) * (size_t)F);
    c.cnt = c.pts + al256(sizeof(int32_t) * (size_t)P);
    c.feat = c.cnt + 256;
    c.X = c.feat + al256(sizeof(float) * DIN * (size_t)(pc * F));
    c.Y = c.X + al256(sizeof(uint16_t) * DIN * (size_t)(pc * F));
    c.Jf = c.Y + al256(sizeof(float) * 2 * (size_t)(pc * F));
    c.total = c.Jf + al256(sizeof(float) * (size_t)(P * F));
    return c;
}

__global__ void k_iota_i32(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}
}  // namespace

extern "C" rt_status rt_closure_J_workspace(const rt_model* m, const rt_dirset* coarse, int64_t F, size_t solve_bytes,
                                            size_t* bytes) {
    if (!m || !coarse || !bytes || F <= 0) return fail(RT_ERR_ARG, "rt_closure_J_workspace: bad arguments");
    int64_t R1 = 0;
    rt_dirset_info(coarse, &R1, nullptr, nullptr, nullptr);
    *bytes = closure_parts(m->P, R1, F).total + solve_bytes;
    return RT_OK;
}

extern "C" rt_status rt_closure_J(const rt_model* m, const rt_dirset* coarse, const rt_dirset* fine, const float* chi,
                                  const float* eta, int64_t ld, const rt_freq_grid* grid, const double* I_bc,
                                  const rt_mlp* h, float log_bound, float* J, int32_t* flagged, int64_t* n_flagged,
                                  const rt_solve_opts* opts, void* ws, size_t ws_bytes, void* stream) {
    if (!m || !coarse || !fine || !chi || !eta || !grid || !I_bc || !h || !J || !flagged || !n_flagged || !ws)
        return fail(RT_ERR_ARG, "rt_closure_J: NULL argument");
    if (!h->has_norm) return fail(RT_ERR_STATE, "rt_closure_J: the network has no input norm (rt_mlp_set_input_norm)");
    rt_solve_opts o = opts ? *opts : default_solve_opts();
    o.precision = RT_F32;
    int64_t F = 0;
    for (int b = 0; b < grid->n_blocks && grid->len; ++b) F += grid->len[b];
    if (F <= 0 || ld < F || grid->n_blocks < 1 || grid->n_blocks > RT_MAX_FREQ_BLOCKS || !grid->dx)
        return fail(RT_ERR_ARG, "rt_closure_J: bad frequency grid");
    int64_t R1 = 0, n1 = 0;
    rt_dirset_info(coarse, &R1, &n1, nullptr, nullptr);
    if (n1 > 0) return fail(RT_ERR_ARG, "rt_closure_J: the coarse set must be shared (uniform)");
    const int64_t P = m->P;
    if (P * F > MAX_SAMPLES) return fail(RT_ERR_UNSUPPORTED, "rt_closure_J: more than 2^31-1 samples");
    const ClosureParts cp = closure_parts(P, R1, F);
    if (ws_bytes <= cp.total) return fail(RT_ERR_CAPACITY, "rt_closure_J: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)ws;
    float* J1 = (float*)(w + cp.J1);
    float* u1 = (float*)(w + cp.u1);
    float* fx = (float*)(w + cp.x);
    int32_t* pts = (int32_t*)(w + cp.pts);
    int32_t* cnt = (int32_t*)(w + cp.cnt);
    float* feat = (float*)(w + cp.feat);
    uint16_t* X = (uint16_t*)(w + cp.X);
    float* Y = (float*)(w + cp.Y);
    float* Jf = (float*)(w + cp.Jf);
    void* solve_ws = w + cp.total;
    const size_t solve_bytes = ws_bytes - cp.total;
    // frequencies in Doppler widths: x = x0[b] + j dx[b] (x0 NULL: centred blocks)
    std::vector<float> hx((size_t)F);
    for (int b = 0, f = 0; b < grid->n_blocks; ++b) {
        const double x0 = grid->x0 ? grid->x0[b] : -0.5 * (grid->len[b] - 1) * grid->dx[b];
        for (int j = 0; j < grid->len[b]; ++j, ++f) hx[(size_t)f] = (float)(x0 + j * grid->dx[b]);
    }
    RT_HIP(hipMemcpyAsync(fx, hx.data(), sizeof(float) * (size_t)F, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_iota_i32, dim3(capped_blocks(nb(P, 256))), dim3(256), 0, s, pts, P);
    RT_HIP(hipGetLastError());
    // coarse solve with its per-pair u
    rt_status st = rt_compute_J(m, coarse, nullptr, P, chi, eta, RT_F32, ld, grid, I_bc, J1, u1, &o, solve_ws,
                                solve_bytes, stream);
    if (st) return st;
    // features -> network -> J = J1 exp(m), flags; points in chunks
    RT_HIP(launch_fill_i32(cnt, 1, 0, s));
    Norm nm;
    std::memcpy(nm.mean, h->mean, sizeof(nm.mean));
    std::memcpy(nm.istd, h->istd, sizeof(nm.istd));
    for (int64_t p0 = 0; p0 < P; p0 += CLOSURE_CHUNK) {
        const int64_t pc = std::min<int64_t>(CLOSURE_CHUNK, P - p0);
        st = rt_closure_features(m, chi, eta, ld, F, fx, J1 + p0 * F, u1 + p0 * R1 * F, R1, pts + p0, pc, feat,
                                 stream);
        if (st) return st;
        hipLaunchKernelGGL(k_normalize, dim3(capped_blocks(nb(pc * F * DIN, 256))), dim3(256), 0, s, feat, pc * F, nm,
                           X);
        RT_HIP(hipGetLastError());
        st = rt_mlp_forward(const_cast<rt_mlp*>(h), X, nullptr, pc * F, Y, 0, nullptr, 0, stream);
        if (st) return st;
        hipLaunchKernelGGL(k_closure_apply, dim3(nb(pc, 256)), dim3(256), 0, s, J1 + p0 * F, Y, pc, F, log_bound,
                           J + p0 * F, flagged, cnt, p0);
        RT_HIP(hipGetLastError());
    }
    int32_t hn = 0;
    RT_HIP(hipMemcpyAsync(&hn, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    *n_flagged = hn;
    if (hn == 0) return RT_OK;
    // the fallback: the plain solve with the fine set at the flagged points, merged into J
    st = rt_compute_J(m, fine, flagged, hn, chi, eta, RT_F32, ld, grid, I_bc, Jf, nullptr, &o, solve_ws, solve_bytes,
                      stream);
    if (st) return st;
    hipLaunchKernelGGL(k_closure_merge, dim3(capped_blocks(nb((int64_t)hn * F, 256))), dim3(256), 0, s, Jf, flagged,
                       (int64_t)hn, F, P, J, error_word());
    RT_HIP(hipGetLastError());
    return RT_OK;
}
