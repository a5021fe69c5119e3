// MLP surrogate of the property path (paper, Section 4): BF16 matrix-core kernels.
//
// Network: 10 -> 256 -> 256 -> 256 -> 256 -> 6, GELU after each hidden layer, L1 loss.
//
// Inference / training forward: one fused kernel.  Cells are the N dimension of
// v_mfma_f32_32x32x16_bf16 (32 cells per wave) and features the M and K dimensions: the
// 32x32 FP32 accumulator of a 32-feature output block holds, in each lane, 16 features of
// one cell, which are exactly the 2 x 8 bf16 values that lane contributes to two K blocks
// of the next layer's B operand.  Activations therefore never leave registers; the next
// layer's weights are stored with the matching permutation of their input index.  The 8
// waves of a workgroup share each layer's weights, staged once per 256-cell tile in LDS
// (rows padded by 16 bytes so that the lanes reading consecutive rows hit distinct banks);
// a 32-row A fragment feeds 32 cells, twice the reuse of the 16x16 shape, which halves the
// LDS traffic per matrix-core operation.  GELU (tanh form, hardware exp2 and reciprocal)
// and the bias are applied in FP32 on the accumulators, then packed to bf16 with
// v_cvt_pk_bf16_f32 (round to nearest even).
//
// Backward: dH = dZ W with the GELU derivative fused in the epilogue (64x64 tiles on the
// 16x16x32 MFMA, W kept transposed so both operands are contiguous along K), dW = dZ^T H on
// the 32x32x16 MFMA with both operands k-major (split over the batch with a fixed-order
// reduction: training is deterministic and resumable bit for bit), column sums for the
// biases, Adam on FP32 master weights.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "props_internal.hpp"
#include "trace.hpp"

namespace props {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short bf16_t;  // storage type of a bfloat16

constexpr int NIN = PROPS_DNN_IN, NOUT = PROPS_DNN_OUT, HID = PROPS_DNN_HIDDEN, NL = PROPS_DNN_LAYERS;
constexpr int IN_PAD = 32;     // input columns of the layer-0 weights and of saved inputs
constexpr int OUT_PAD = 16;    // output rows of the last layer's weights and saved outputs
constexpr int HROW = HID + 8;  // bf16 per weight row in the fused layout (528 B)
constexpr int FK0 = 16;        // layer-0 K in the fused layout: one 16-deep K block
constexpr int IROW = FK0 + 8;  // bf16 per layer-0 fused row (48 B)
constexpr int FOUT_ROWS = 32;  // last layer padded to one 32-row output block
constexpr int FWD_WAVES = 8;
constexpr int FWD_THREADS = FWD_WAVES * 64;
constexpr int CELLS_PER_WAVE = 32;
constexpr int TILE_CELLS = FWD_WAVES * CELLS_PER_WAVE;   // 256
constexpr int MAX_BATCH = 65536;
constexpr int SPLITW = 128;    // batch splits of the weight-gradient GEMMs (32: 89M, 64: 106M,
                               // 128: 115M, 256: 108M training samples/s)
// LDS fragment prefetch distance of the hidden layers, in matrix-core steps (1 measured
// 6 % slower on the 2^22-cell inference; 2 to 6 alike)
constexpr int FPF = 3;
// Outputs of the (P, T, Y) surrogate trained on their logarithm: rho, cp, mu, lambda
// (bits 0, 2, 4, 5; h and c cross or approach zero and stay linear).
constexpr unsigned kPTYLogMask = 0x35u;

// padded (out, in) of each weight layer and its offsets in the FP32 master vector
__host__ __device__ constexpr int lout(int l) { return l == 0 ? HID : (l == NL - 1 ? OUT_PAD : HID); }
__host__ __device__ constexpr int lin(int l) { return l == 0 ? IN_PAD : HID; }
__host__ __device__ constexpr int lrow(int l) { return l == 0 ? IROW : HROW; }
// true (unpadded) shapes
__host__ __device__ constexpr int tout(int l) { return l == NL - 1 ? NOUT : HID; }
__host__ __device__ constexpr int tin(int l) { return l == 0 ? NIN : HID; }

// offsets of each layer in the FP32 master vector (W then b), the fused bf16 layout and
// the natural bf16 layout
__host__ __device__ constexpr size_t w_off(int l) { return l == 0 ? 0 : w_off(l - 1) + (size_t)lout(l - 1) * lin(l - 1) + lout(l - 1); }
__host__ __device__ constexpr size_t b_off(int l) { return w_off(l) + (size_t)lout(l) * lin(l); }
// rows of each layer in the fused layout (the last layer padded to a 32-row block)
__host__ __device__ constexpr int frows(int l) { return l == NL - 1 ? FOUT_ROWS : lout(l); }
__host__ __device__ constexpr size_t f_off(int l) { return l == 0 ? 0 : f_off(l - 1) + (size_t)frows(l - 1) * lrow(l - 1); }
__host__ __device__ constexpr size_t n_off(int l) { return l == 0 ? 0 : n_off(l - 1) + (size_t)lout(l - 1) * lin(l - 1); }
struct Layout {
    static constexpr size_t total = w_off(NL);
    static constexpr size_t ftotal = f_off(NL);
    static constexpr size_t nattotal = n_off(NL);
    __host__ __device__ static constexpr size_t w(int l) { return w_off(l); }
    __host__ __device__ static constexpr size_t b(int l) { return b_off(l); }
    __host__ __device__ static constexpr size_t f(int l) { return f_off(l); }
    __host__ __device__ static constexpr size_t nat(int l) { return n_off(l); }
};
using kLay = Layout;

// Largest fused layer in bytes (the LDS staging buffer).
constexpr int LDS_BYTES = HID * HROW * 2;   // 135168

// ------------------------------------------------------------------ small device helpers
// two floats -> two bf16 (round to nearest even; v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ unsigned pack_bf16x2(float a, float b)
{
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    bf2 v = __builtin_convertvector((f2){a, b}, bf2);
    return __builtin_bit_cast(unsigned, v);
}

__device__ __forceinline__ bf16_t to_bf16(float a) { return (bf16_t)(pack_bf16x2(a, 0.0f) & 0xffffu); }

__device__ __forceinline__ float bf16_to_f(bf16_t h) { return __builtin_bit_cast(float, (unsigned)h << 16); }

// k-slot of input feature i (i >= 0) in the fused layout of a layer after a hidden one: the
// 32x32 accumulator gives lane half h the features 8q + 4h + (0..3) of a block, q = 0..3,
// and its values 8c..8c+7 form K block 2 ob + c, so within each 16-feature block r = i % 16
// sits at slot 8 ((r >> 2) & 1) + 4 (r >> 3) + (r & 3): bits 2 and 3 of r swap.
__host__ __device__ constexpr int kslot(int i)
{
    return (i & ~15) | (((i >> 2) & 1) << 3) | (((i >> 3) & 1) << 2) | (i & 3);
}

// GELU, tanh form of Hendrycks & Gimpel: x * sigmoid(2 sqrt(2/pi) (x + 0.044715 x^3)),
// with exp2 and reciprocal on the transcendental unit.
constexpr float kG0 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;  // -2 sqrt(2/pi) log2(e)
constexpr float kG1 = kG0 * 0.044715f;
__device__ __forceinline__ float gelu_f(float x)
{
    float t = x * __builtin_fmaf(kG1, x * x, kG0);
    float e = __builtin_amdgcn_exp2f(t);
    return x * __builtin_amdgcn_rcpf(1.0f + e);
}

// d/dx of gelu_f
__device__ __forceinline__ float gelu_grad_f(float x)
{
    float x2 = x * x;
    float t = x * __builtin_fmaf(kG1, x2, kG0);
    float e = __builtin_amdgcn_exp2f(t);
    float s = __builtin_amdgcn_rcpf(1.0f + e);           // sigmoid(2u)
    float up = 2.0f * 0.7978845608028654f * (1.0f + 3.0f * 0.044715f * x2);   // 2 u'(x)
    return s + x * s * (1.0f - s) * up;
}

__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// sample index of training row i in epoch permutation (a odd/coprime, c offset)
__device__ __forceinline__ int64_t perm_index(int64_t i, uint64_t a, uint64_t c, int64_t n)
{
    return (int64_t)(((unsigned __int128)a * (uint64_t)i + c) % (uint64_t)n);
}

// ------------------------------------------------------------------ fused forward
struct FwdArgs {
    // inference inputs (SoA doubles) ...
    const double *P, *T, *Y;
    // ... or training inputs (feature-major float [10][nx]) with the epoch permutation
    const float *X;
    int64_t nx;
    uint64_t pa, pc;
    int64_t row0;        // first permuted row of this batch
    int64_t n;           // cells (rows) this launch covers
    int64_t ldy;         // inference: element stride between the species rows of Y (>= n)
    const bf16_t *Wf;    // fused-layout weights of all layers
    const float *bias;   // FP32 master vector (biases read from their offsets)
    const double *in_lo, *in_inv;   // [10] input box
    const double *out_lo, *out_rng; // [6] target box
    unsigned logmask;               // bit j: output j was trained on its logarithm
    // ... or inference on raw feature-major inputs [10][n], outputs [6][n]
    const double *Xd;
    double *Yd;
    // inference outputs
    double *orho, *oh, *ocp, *oc, *omu, *olam;
    uint8_t *status;
    int *fb_idx, *fb_count;         // fallback list (cells outside the box / non-physical)
    // training saves
    bf16_t *h0;          // [n][32]
    float *z[4];         // [n][256] pre-activations of the hidden layers
    bf16_t *h[4];        // [n][256] activations
    float *y;            // [n][16] output layer
};

// Stage one fused layer (rows x row-stride bf16, a multiple of 16 bytes) into LDS with
// global_load_lds_dwordx4: each lane's 16 bytes go straight to LDS base + 16 lane, without
// passing through registers; one 1 KB chunk per wave and instruction.
__device__ __forceinline__ void stage(unsigned char *lds, const bf16_t *src, int bytes)
{
    const uint4 *s = reinterpret_cast<const uint4 *>(src);
    const int n16 = bytes / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = wave; c * 64 < n16; c += FWD_WAVES) {
        const int i = c * 64 + lane;
        if (i < n16)
            __builtin_amdgcn_global_load_lds((const void *)(s + i),
                                             (__attribute__((address_space(3))) void *)(lds + c * 1024), 16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);   // this wave's loads have landed (the caller's barrier does the rest)
}

__device__ __forceinline__ bf16x8 lds_frag(const unsigned char *lds, int row, int rowlen, int slot)
{
    return *reinterpret_cast<const bf16x8 *>(lds + ((size_t)row * rowlen + slot) * 2);
}

// Bias-initialised accumulator of output block ob: lane half h holds rows 8q + 4h + (0..3);
// only the first nq row groups exist (the last layer has 16 bias entries, nq = 2).
__device__ __forceinline__ f32x16 bias_block(const float *bias, int ob, int h, int nq = 4)
{
    f32x16 c;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const f32x4 b = (q < nq) ? *reinterpret_cast<const f32x4 *>(bias + 32 * ob + 8 * q + 4 * h) : f32x4{};
        c[4 * q + 0] = b[0];
        c[4 * q + 1] = b[1];
        c[4 * q + 2] = b[2];
        c[4 * q + 3] = b[3];
    }
    return c;
}

// Training saves of one 32-feature block of layer l: pre-activations z (FP32) and the
// packed bf16 activations p (8 pairs), in natural feature order [cell][256].
__device__ __forceinline__ void save_block(const FwdArgs &a, int l, int64_t cell, int ob, int h,
                                           const f32x16 &z, const unsigned *p)
{
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int64_t off = cell * HID + 32 * ob + 8 * q + 4 * h;
        *reinterpret_cast<f32x4 *>(a.z[l] + off) = f32x4{z[4 * q], z[4 * q + 1], z[4 * q + 2], z[4 * q + 3]};
        *reinterpret_cast<uint2 *>(a.h[l] + off) = make_uint2(p[2 * q], p[2 * q + 1]);
    }
}
template <bool TRAIN>
__global__ __launch_bounds__(FWD_THREADS, 1) void mlp_fwd_kernel(FwdArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5;         // lane half: K slots 8h..8h+7 (A, B); rows 8q + 4h.. (C)
    const int col = lane & 31;       // cell within the wave's 32-cell block (B, C); A row
    const int64_t ntiles = (a.n + TILE_CELLS - 1) / TILE_CELLS;

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        bf16x8 act[16];              // B operand: one bf16x8 per 16-deep K block
#pragma unroll
        for (int kb = 0; kb < 16; kb++) act[kb] = bf16x8{};
        const int64_t cell = tile * TILE_CELLS + wave * CELLS_PER_WAVE + col;
        const bool live = cell < a.n;
        uint8_t flag = 0;
        // ---- inputs -> scaled bf16 B operand of layer 0 (half 0: features 0..7, half 1: 8, 9)
        {
            float xs[8];
#pragma unroll
            for (int j = 0; j < 8; j++) xs[j] = 0.0f;
            if (live) {
                double raw[NIN];
                if (TRAIN) {
                    const int64_t sidx = perm_index(a.row0 + cell, a.pa, a.pc, a.nx);
#pragma unroll
                    for (int f = 0; f < NIN; f++) raw[f] = (double)a.X[(int64_t)f * a.nx + sidx];
                } else if (a.Xd) {
#pragma unroll
                    for (int f = 0; f < NIN; f++) raw[f] = a.Xd[(int64_t)f * a.n + cell];
                } else {
                    raw[0] = a.P[cell];
                    raw[1] = a.T[cell];
#pragma unroll
                    for (int f = 0; f < NIN - 2; f++) raw[2 + f] = a.Y[(int64_t)f * a.ldy + cell];
                }
                if (h == 0) {
#pragma unroll
                    for (int j = 0; j < 8; j++) xs[j] = (float)((raw[j] - a.in_lo[j]) * a.in_inv[j]);
                } else {
#pragma unroll
                    for (int j = 0; j < NIN - 8; j++) xs[j] = (float)((raw[8 + j] - a.in_lo[8 + j]) * a.in_inv[8 + j]);
                }
                if (!TRAIN && !a.Xd && h == 0) {
                    // training box (the hull) and physical sanity of the whole cell
                    bool out = false, bad = !(raw[0] > 0.0) || !(raw[1] > 0.0);
                    double sy = 0.0;
#pragma unroll
                    for (int f = 0; f < NIN; f++) {
                        // a feature constant in the training data (in_inv = 0) scales to 0
                        // for the network, but the box still holds only that one value
                        const double d = raw[f] - a.in_lo[f];
                        const double sc = d * a.in_inv[f];
                        out |= (a.in_inv[f] != 0.0) ? !(sc >= -1e-9 && sc <= 1.0 + 1e-9)
                                                    : !(fabs(d) <= 1e-9 * fmax(1.0, fabs(a.in_lo[f])));
                    }
#pragma unroll
                    for (int f = 2; f < NIN; f++) {
                        bad |= !(raw[f] >= -1e-12);
                        sy += raw[f];
                    }
                    bad |= !(fabs(sy - 1.0) <= 1e-6);
                    flag = (out || bad) ? 1 : 0;
                }
            }
            unsigned p[4];
#pragma unroll
            for (int j = 0; j < 4; j++) p[j] = pack_bf16x2(xs[2 * j], xs[2 * j + 1]);
            act[0] = __builtin_bit_cast(bf16x8, *reinterpret_cast<uint4 *>(p));
            if (TRAIN && live) {
                // saved inputs keep IN_PAD columns; 16..31 stay zero from allocation
                *reinterpret_cast<uint4 *>(a.h0 + cell * IN_PAD + 8 * h) = *reinterpret_cast<uint4 *>(p);
            }
        }

        // ---- hidden layers 0..3 (GELU)
#pragma unroll 1
        for (int l = 0; l < NL - 1; l++) {
            __syncthreads();   // previous layer done with the LDS buffer
            const int rowlen = lrow(l);
            stage(lds, a.Wf + kLay::f(l), frows(l) * rowlen * 2);
            __syncthreads();
            const float *bias = a.bias + kLay::b(l);
            bf16x8 nxt[16];
            if (l == 0) {
                // one 16-deep K block: eight single MFMAs, then GELU
#pragma unroll
                for (int ob = 0; ob < 8; ob++) {
                    const bf16x8 a0 = lds_frag(lds, ob * 32 + col, rowlen, 8 * h);
                    const f32x16 z = mfma32(a0, act[0], bias_block(bias, ob, h));
                    unsigned p[8];
#pragma unroll
                    for (int q = 0; q < 8; q++) p[q] = pack_bf16x2(gelu_f(z[2 * q]), gelu_f(z[2 * q + 1]));
                    nxt[2 * ob] = __builtin_bit_cast(bf16x8, make_uint4(p[0], p[1], p[2], p[3]));
                    nxt[2 * ob + 1] = __builtin_bit_cast(bf16x8, make_uint4(p[4], p[5], p[6], p[7]));
                    if (TRAIN && live) save_block(a, 0, cell, ob, h, z, p);
                }
            } else {
                // One 32-row output block per step; the GELU of block ob - 1 is interleaved
                // with the matrix-core work of block ob (one value per K block), so that the
                // vector and matrix units of a SIMD work at the same time.
                // The 128 matrix-core steps of the layer (8 blocks x 16 K blocks) read their
                // A fragments from LDS FPF steps ahead, across block boundaries.
                const auto frag = [&](int st) {
                    return lds_frag(lds, (st >> 4) * 32 + col, rowlen, (st & 15) * 16 + 8 * h);
                };
                bf16x8 ring[FPF];
#pragma unroll
                for (int d = 0; d < FPF; d++) ring[d] = frag(d);
                f32x16 pz = {};
#pragma unroll
                for (int ob = 0; ob <= 8; ob++) {
                    f32x16 acc = {};
                    unsigned pg[8];
                    float gv[16];
                    if (ob < 8) acc = bias_block(bias, ob, h);
#pragma unroll
                    for (int kb = 0; kb < 16; kb++) {
                        if (ob < 8) {
                            const int st = ob * 16 + kb;
                            const bf16x8 cur = ring[st % FPF];
                            if (st + FPF < 128) ring[st % FPF] = frag(st + FPF);
                            acc = mfma32(cur, act[kb], acc);
                        }
                        if (ob > 0) {
                            gv[kb] = gelu_f(pz[kb]);
                            if (kb & 1) pg[kb >> 1] = pack_bf16x2(gv[kb - 1], gv[kb]);
                        }
                        if (ob > 0 && ob < 8) {
                            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
                            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
                            __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);   // VALU
                        } else {
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                    if (ob > 0) {
                        const int pb = ob - 1;
                        nxt[2 * pb] = __builtin_bit_cast(bf16x8, make_uint4(pg[0], pg[1], pg[2], pg[3]));
                        nxt[2 * pb + 1] = __builtin_bit_cast(bf16x8, make_uint4(pg[4], pg[5], pg[6], pg[7]));
                        if (TRAIN && live) save_block(a, l, cell, pb, h, pz, pg);
                    }
                    if (ob < 8) pz = acc;
                }
            }
#pragma unroll
            for (int kb = 0; kb < 16; kb++) act[kb] = nxt[kb];
        }
        // ---- output layer (linear), outside the loop so that its double-precision
        // epilogue does not share the register budget of the hidden layers
        {
            constexpr int l = NL - 1;
            __syncthreads();
            const int rowlen = lrow(l);
            stage(lds, a.Wf + kLay::f(l), frows(l) * rowlen * 2);
            __syncthreads();
            const float *bias = a.bias + kLay::b(l);
            {
                f32x16 acc = bias_block(bias, 0, h, OUT_PAD / 8);   // rows 16..31: padding
#pragma unroll
                for (int kb = 0; kb < 16; kb++) {
                    const bf16x8 a0 = lds_frag(lds, col, rowlen, kb * 16 + 8 * h);
                    acc = mfma32(a0, act[kb], acc);
                }
                if (live) {
                    if (TRAIN) {
                        // rows 8q + 4h + (0..3) for q = 0, 1 are the 16 saved outputs
#pragma unroll
                        for (int q = 0; q < 2; q++)
                            *reinterpret_cast<f32x4 *>(a.y + cell * OUT_PAD + 8 * q + 4 * h) =
                                f32x4{acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]};
                    } else if (a.Yd) {
                        // feature-major outputs in target units: lanes of half 0 hold rows
                        // 0..3, half 1 rows 4, 5; the rows flagged in logmask were trained
                        // on their logarithm
                        const int j0 = 4 * h;
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int j = j0 + v;
                            if (j < NOUT) {
                                const double y = a.out_lo[j] + (double)acc[v] * a.out_rng[j];
                                a.Yd[(int64_t)j * a.n + cell] = (a.logmask >> j & 1u) ? exp(y) : y;
                            }
                        }
                    } else if (h == 0) {
                        // rows 0..3: rho, h, cp, c
                        if (a.orho) a.orho[cell] = exp(a.out_lo[0] + (double)acc[0] * a.out_rng[0]);
                        if (a.oh) a.oh[cell] = a.out_lo[1] + (double)acc[1] * a.out_rng[1];
                        if (a.ocp) a.ocp[cell] = exp(a.out_lo[2] + (double)acc[2] * a.out_rng[2]);
                        if (a.oc) a.oc[cell] = a.out_lo[3] + (double)acc[3] * a.out_rng[3];
                    } else {
                        // rows 4, 5: mu, lambda
                        if (a.omu) a.omu[cell] = exp(a.out_lo[4] + (double)acc[0] * a.out_rng[4]);
                        if (a.olam) a.olam[cell] = exp(a.out_lo[5] + (double)acc[1] * a.out_rng[5]);
                    }
                }
            }
        }
        if (!TRAIN) {
            // status and fallback list (lanes of half 0 own their cell)
            const bool mine = live && h == 0;
            const bool f = mine && flag;
            if (mine && a.status) a.status[cell] = f ? PROPS_ST_OUT_OF_HULL : 0;
            if (a.fb_idx) {
                const unsigned long long bal = __ballot(f);
                const int cnt = __popcll(bal);
                int base = 0;
                if (cnt) {
                    const int first = __builtin_ctzll(bal);
                    if (lane == first) base = atomicAdd(a.fb_count, cnt);
                    base = __shfl(base, first);
                    if (f) a.fb_idx[base + __popcll(bal & ((1ull << lane) - 1))] = (int)cell;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ input-gradient GEMM
// D[m][n] = bf16( (sum_k A[m][k] B[n][k]) gelu'(Z[m][n]) ): dz_{l-1} = (dz_l W_l) * GELU'(z_{l-1})
// with A = dz_l (rows = batch, K = the layer's outputs) and B = W_l transposed ([in][out]),
// both contiguous along K.  64 x 64 tiles, K in steps of 32 staged in LDS with 16-byte
// stores, 4 waves of 2 x 2 v_mfma_f32_16x16x32_bf16 blocks.  M, N, K, lda, ldb multiples of 8.
// (An LDS-free variant with 16-byte fragment loads straight from global memory, cells on
// either MFMA side, measured 1.5-2x slower.)
struct GemmArgs {
    int M, N, K;
    const bf16_t *A;
    int lda;
    const bf16_t *B;
    int ldb;
    bf16_t *Cb;
    int ldc;
    const float *Z;
    int ldz;
};

__global__ __launch_bounds__(256) void gemm_dh_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) bf16_t As[64][40];
    __shared__ __attribute__((aligned(16))) bf16_t Bs[64][40];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += 32) {
        // A tile (64 m x 32 k) -> As[m][k]; B tile (64 n x 32 k) -> Bs[n][k]
        const int r = t >> 2, k8 = (t & 3) * 8;
        uint4 va = make_uint4(0, 0, 0, 0), vb = make_uint4(0, 0, 0, 0);
        if (m0 + r < g.M && k0 + k8 < g.K) va = *reinterpret_cast<const uint4 *>(g.A + (int64_t)(m0 + r) * g.lda + k0 + k8);
        if (n0 + r < g.N && k0 + k8 < g.K) vb = *reinterpret_cast<const uint4 *>(g.B + (int64_t)(n0 + r) * g.ldb + k0 + k8);
        *reinterpret_cast<uint4 *>(&As[r][k8]) = va;
        *reinterpret_cast<uint4 *>(&Bs[r][k8]) = vb;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&As[wm * 32 + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
            for (int j = 0; j < 2; j++) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&Bs[wn * 32 + j * 16 + (lane & 15)][8 * (lane >> 4)]);
                acc[i][j] = mfma16(av, bv, acc[i][j]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int n = n0 + wn * 32 + j * 16 + (lane & 15);
                if (m < g.M && n < g.N) {
                    const float d = acc[i][j][r] * gelu_grad_f(g.Z[(int64_t)m * g.ldz + n]);
                    g.Cb[(int64_t)m * g.ldc + n] = to_bf16(d);
                }
            }
}

// ------------------------------------------------------------------ training helpers
// L1 loss gradient on the scaled targets: dz[i][j] = sign(y - t) / (n_rows * 6) for j < 6.
// Per-block partial sums of |y - t| go to part[blockIdx.x] (fixed-order reduction later).
__global__ __launch_bounds__(256) void l1_grad_kernel(const float *y, const float *Yraw, int64_t nx,
                                                      uint64_t pa, uint64_t pc, int64_t row0, int n,
                                                      const double *out_lo, const double *out_inv,
                                                      unsigned logmask, bf16_t *dz, float *part)
{
    __shared__ float red[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    float s = 0.f;
    if (i < n) {
        const int64_t sidx = perm_index(row0 + i, pa, pc, nx);
        const float scale = 1.0f / ((float)n * NOUT);
#pragma unroll
        for (int j = 0; j < OUT_PAD; j++) {
            float d = 0.f;
            if (j < NOUT) {
                double tr = (double)Yraw[(int64_t)j * nx + sidx];
                if (logmask >> j & 1u) tr = log(tr);
                const float t = (float)((tr - out_lo[j]) * out_inv[j]);
                const float diff = y[(int64_t)i * OUT_PAD + j] - t;
                s += fabsf(diff);
                d = (diff > 0.f) ? scale : ((diff < 0.f) ? -scale : 0.f);
            }
            dz[(int64_t)i * OUT_PAD + j] = to_bf16(d);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[i] = sum_s part[s * stride + i] in order s = 0..S-1 (deterministic split-K reduction),
// with the result written to dst[i] (gradient of a weight matrix).
__global__ void reduce_partials_kernel(const float *part, int S, int64_t stride, int64_t count, float *dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.f;
    int k = 0;
    for (; k + 8 <= S; k += 8) {   // eight partials in flight, summed in order
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) v[j] = part[(k + j) * stride + i];
#pragma unroll
        for (int j = 0; j < 8; j++) s += v[j];
    }
    for (; k < S; k++) s += part[k * stride + i];
    dst[i] = s;
}

// Column sums of a bf16 [n][ncol] matrix (ncol a multiple of 8, at most 256): block p sums
// rows [p*rows, ...) into part[p][col].  Thread (g, c8) adds the 8 columns 8 c8.. of rows
// r0 + g, r0 + g + G, ... with 16-byte loads; the G row groups are then combined in a fixed
// order, so the result is deterministic.
__global__ __launch_bounds__(256) void colsum_partial_kernel(const bf16_t *dz, int n, int ncol, int rows, float *part)
{
    __shared__ float red[256 * 8];
    const int cg = ncol / 8;                  // 16-byte column groups per row
    const int G = 256 / cg;                   // row groups per block
    const int g = threadIdx.x / cg, c8 = threadIdx.x % cg;
    const int r0 = blockIdx.x * rows, r1 = min(n, r0 + rows);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (g < G) {
        for (int r = r0 + g; r < r1; r += G) {
            const uint4 v = *reinterpret_cast<const uint4 *>(dz + (int64_t)r * ncol + 8 * c8);
            const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                acc[2 * j] += __builtin_bit_cast(float, w[j] << 16);
                acc[2 * j + 1] += __builtin_bit_cast(float, w[j] & 0xffff0000u);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 8; j++) red[threadIdx.x * 8 + j] = acc[j];
    __syncthreads();
    if (threadIdx.x < ncol) {
        const int c = threadIdx.x;
        float s = 0.f;
        for (int q = 0; q < G; q++) s += red[(q * cg + c / 8) * 8 + (c % 8)];
        part[blockIdx.x * ncol + c] = s;
    }
}

// dst[c] = sum_p part[p][c] in the order p = 0, 1, ... (one thread per column, eight
// partial rows loaded at a time)
// dst[c] = sum over the P partial rows of column c.  A block takes 64 columns; its four
// wave-sized groups sum every fourth row (eight loads in flight), then one group adds the
// four group sums in a fixed order, so the result is the same bits on every run.
__global__ __launch_bounds__(256) void sum_rows_kernel(const float *part, int P, int ncol, float *dst)
{
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63);
    const int g = threadIdx.x >> 6;
    float s = 0.f;
    if (c < ncol) {
        int p = g;
        for (; p + 28 < P; p += 32) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; j++) v[j] = part[(int64_t)(p + 4 * j) * ncol + c];
#pragma unroll
            for (int j = 0; j < 8; j++) s += v[j];
        }
        for (; p < P; p += 4) s += part[(int64_t)p * ncol + c];
    }
    red[g][threadIdx.x & 63] = s;
    __syncthreads();
    if (g == 0 && c < ncol) dst[c] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

__global__ void adam_kernel(float *w, const float *gr, float *m, float *v, int64_t n, float lr,
                            float b1, float b2, float eps, float bc1, float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// FP32 master -> bf16 transposed [in][out] (the B operand of dz W, contiguous along its K
// = out) and fused (row-padded, k-permuted) layouts.
__global__ void convert_weights_kernel(const float *master, bf16_t *nat, bf16_t *fused)
{
    const int l = blockIdx.y;
    const int rows = lout(l), cols = lin(l), rowlen = lrow(l);
    const int64_t cnt = (int64_t)rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)(e / cols), i = (int)(e % cols);
        const float wv = master[kLay::w(l) + e];
        const bf16_t b = to_bf16(wv);
        nat[kLay::nat(l) + (int64_t)i * rows + o] = b;   // transposed: [in][out]
        // layer 0 keeps the natural input order in its one 16-deep K block (inputs >= 16
        // are padding); later layers take the permutation of the accumulator layout
        if (l == 0 && i >= FK0) continue;
        const int slot = (l == 0) ? i : kslot(i);
        fused[kLay::f(l) + (int64_t)o * rowlen + slot] = b;
    }
}

__global__ void fill_int_kernel(int *p, int v) { *p = v; }

__global__ void fill_float_kernel(float *p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// feature-wise min/max of a [nf][n] float array (transform: log for the flagged rows)
__global__ void minmax_partial_kernel(const float *X, int64_t n, int nf, unsigned logmask, int64_t per, double *part)
{
    const int f = blockIdx.y;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(n, r0 + per);
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        double x = X[(int64_t)f * n + r];
        if (logmask >> f & 1u) x = log(x);
        lo = fmin(lo, x);
        hi = fmax(hi, x);
    }
    __shared__ double sl[256], sh[256];
    sl[threadIdx.x] = lo;
    sh[threadIdx.x] = hi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + w]);
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[((int64_t)f * gridDim.x + blockIdx.x) * 2] = sl[0];
        part[((int64_t)f * gridDim.x + blockIdx.x) * 2 + 1] = sh[0];
    }
}

// ------------------------------------------------------------------ splitmix64 (Steele, Lea & Flood 2014)
static uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double u01(uint64_t &s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace props

using namespace props;

// ------------------------------------------------------------------ the handle
struct props_dnn_s {
    int device = 0;
    float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;   // device FP32
    bf16_t *nat = nullptr, *fused = nullptr;
    double *scal = nullptr;        // device: in_lo[10], in_inv[10], out_lo[6], out_rng[6], out_inv[6]
    double in_lo[NIN], in_hi[NIN], out_lo[NOUT], out_hi[NOUT];
    unsigned logmask = kPTYLogMask;   // outputs trained on their logarithm
    int64_t step = 0;
    int epoch = 0;
    // forward/backward scratch for one batch
    bf16_t *h0 = nullptr, *hs[4] = {}, *dz = nullptr, *dz2 = nullptr, *dzo = nullptr;
    float *zs[4] = {}, *y = nullptr, *part = nullptr, *lpart = nullptr, *cpart = nullptr;
    int *fb_idx = nullptr, *fb_count = nullptr;
    int64_t fb_cap = 0;
};

namespace props {

static int upload_scalers(props_dnn_s *d)
{
    double h[NIN * 2 + NOUT * 3];
    for (int f = 0; f < NIN; f++) {
        h[f] = d->in_lo[f];
        const double r = d->in_hi[f] - d->in_lo[f];
        h[NIN + f] = (r > 0) ? 1.0 / r : 0.0;
    }
    for (int j = 0; j < NOUT; j++) {
        const double r = d->out_hi[j] - d->out_lo[j];
        h[2 * NIN + j] = d->out_lo[j];
        h[2 * NIN + NOUT + j] = r;
        h[2 * NIN + 2 * NOUT + j] = (r > 0) ? 1.0 / r : 0.0;
    }
    PROPS_HIP_TRY(hipMemcpy(d->scal, h, sizeof(h), hipMemcpyHostToDevice));
    return PROPS_OK;
}

static int refresh_weights(props_dnn_s *d, hipStream_t s)
{
    hipLaunchKernelGGL(convert_weights_kernel, dim3(64, NL), dim3(256), 0, s, d->master, d->nat, d->fused);
    PROPS_HIP_TRY(hipGetLastError());
    return PROPS_OK;
}

template <typename T>
static int dalloc(T **p, size_t count)
{
    hipError_t e = hipMalloc((void **)p, sizeof(T) * count);
    if (e != hipSuccess) return fail(PROPS_ENOMEM, "hipMalloc(%zu): %s", sizeof(T) * count, hipGetErrorString(e));
    return PROPS_OK;
}

static void free_dnn(props_dnn_s *d)
{
    void *ps[] = {d->master, d->grad, d->m, d->v, d->nat, d->fused, d->scal, d->h0, d->dz, d->dz2, d->dzo,
                  d->y, d->part, d->lpart, d->cpart, d->fb_idx, d->fb_count,
                  d->hs[0], d->hs[1], d->hs[2], d->hs[3], d->zs[0], d->zs[1], d->zs[2], d->zs[3]};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete d;
}

static int alloc_dnn(props_dnn_s *d)
{
    int rc;
    const size_t P = kLay::total;
    if ((rc = dalloc(&d->master, P)) || (rc = dalloc(&d->grad, P)) || (rc = dalloc(&d->m, P)) ||
        (rc = dalloc(&d->v, P)) || (rc = dalloc(&d->nat, kLay::nattotal)) ||
        (rc = dalloc(&d->fused, kLay::ftotal)) || (rc = dalloc(&d->scal, (size_t)NIN * 2 + NOUT * 3)) ||
        (rc = dalloc(&d->fb_count, 1)))
        return rc;
    PROPS_HIP_TRY(hipMemset(d->grad, 0, P * sizeof(float)));
    PROPS_HIP_TRY(hipMemset(d->m, 0, P * sizeof(float)));
    PROPS_HIP_TRY(hipMemset(d->v, 0, P * sizeof(float)));
    PROPS_HIP_TRY(hipMemset(d->fused, 0, kLay::ftotal * sizeof(bf16_t)));
    return PROPS_OK;
}

static int ensure_train_scratch(props_dnn_s *d)
{
    if (d->h0) return PROPS_OK;
    int rc;
    const size_t B = MAX_BATCH;
    if ((rc = dalloc(&d->h0, B * IN_PAD)) || (rc = dalloc(&d->dz, B * HID)) || (rc = dalloc(&d->dz2, B * HID)) ||
        (rc = dalloc(&d->dzo, B * OUT_PAD)) || (rc = dalloc(&d->y, B * OUT_PAD)) ||
        (rc = dalloc(&d->part, (size_t)SPLITW * HID * HID)) || (rc = dalloc(&d->lpart, (size_t)B / 256 + 64)) ||
        (rc = dalloc(&d->cpart, (size_t)256 * HID)))
        return rc;
    // the forward writes input columns 0..15 of the saved inputs; 16..31 stay zero
    PROPS_HIP_TRY(hipMemset(d->h0, 0, sizeof(bf16_t) * B * IN_PAD));
    for (int l = 0; l < 4; l++)
        if ((rc = dalloc(&d->hs[l], B * HID)) || (rc = dalloc(&d->zs[l], B * HID))) return rc;
    return PROPS_OK;
}

static int fwd_grid(int64_t n)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    const int64_t tiles = (n + TILE_CELLS - 1) / TILE_CELLS;
    return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, cus));
}

static std::once_flag g_lds_once;
static hipError_t g_lds_err = hipSuccess;
static int launch_fwd(bool train, const FwdArgs &a, hipStream_t s)
{
    std::call_once(g_lds_once, [] {
        g_lds_err = hipFuncSetAttribute((const void *)mlp_fwd_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BYTES);
        if (g_lds_err == hipSuccess)
            g_lds_err = hipFuncSetAttribute((const void *)mlp_fwd_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BYTES);
    });
    if (g_lds_err != hipSuccess) return fail(PROPS_EHIP, "hipFuncSetAttribute(LDS %d B): %s", LDS_BYTES, hipGetErrorString(g_lds_err));
    const int grid = fwd_grid(a.n);
    if (train) hipLaunchKernelGGL(mlp_fwd_kernel<true>, dim3(grid), dim3(FWD_THREADS), LDS_BYTES, s, a);
    else hipLaunchKernelGGL(mlp_fwd_kernel<false>, dim3(grid), dim3(FWD_THREADS), LDS_BYTES, s, a);
    PROPS_HIP_TRY(hipGetLastError());
    return PROPS_OK;
}

// Weight gradient C_z[m][n] = sum_{k in split z} A[k][m] B[k][n], with both operands stored
// k-major ([batch][feature] activations and output gradients), on v_mfma_f32_32x32x16_bf16,
// K in steps of 32.  The matrix cores want each lane's eight bf16 consecutive along K, so tiles
// are staged in LDS as bf16 pairs (k even, k odd) per column: a thread reads two k rows of
// eight columns (two 16-byte loads), interleaves them and stores eight pair-dwords; a
// fragment is then four 4-byte LDS reads.  Rows of 136 dwords put the two lane halves of a
// fragment read 32 banks apart.  Double-buffered: the next step's global loads are in
// flight during the current step's MFMAs, one barrier per step.
// A tile of TM x TN outputs per workgroup of 4 waves arranged WAVES_M x (4 / WAVES_M), each
// wave BM x BN blocks of 32 x 32.  Columns at or beyond M (N) read as zero and are not
// written, so the 16-row output layer runs on a 32-row tile.
constexpr int KW_PAD = 8;          // extra pair-dwords per LDS row
__device__ __forceinline__ void kw_interleave(uint4 x, uint4 y, uint4 &lo, uint4 &hi)
{
    // x: row 2kp, y: row 2kp + 1, eight bf16 columns each -> eight (x_j, y_j) pairs
    const unsigned xs[4] = {x.x, x.y, x.z, x.w}, ys[4] = {y.x, y.y, y.z, y.w};
    unsigned d[8];
#pragma unroll
    for (int w = 0; w < 4; w++) {
        d[2 * w] = (xs[w] & 0xffffu) | (ys[w] << 16);
        d[2 * w + 1] = (xs[w] >> 16) | (ys[w] & 0xffff0000u);
    }
    lo = make_uint4(d[0], d[1], d[2], d[3]);
    hi = make_uint4(d[4], d[5], d[6], d[7]);
}

template <int TM, int TN, int WAVES_M>
__global__ __launch_bounds__(256) void gemm_wgrad_kernel(const bf16_t *A, int lda, int M, const bf16_t *B, int ldb,
                                                          int N, int K, int kchunk, float *C, int ldc, int64_t strideC)
{
    constexpr int WAVES_N = 4 / WAVES_M;
    constexpr int BM = TM / WAVES_M / 32, BN = TN / WAVES_N / 32;
    constexpr int CA = TM / 8, CB = TN / 8;   // 16-byte column chunks per k row
    __shared__ __attribute__((aligned(16))) unsigned As[2][16][TM + KW_PAD];
    __shared__ __attribute__((aligned(16))) unsigned Bs[2][16][TN + KW_PAD];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w / WAVES_N, wn = w % WAVES_N;
    const int h = lane >> 5, r = lane & 31;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    // loader work items: (pair row kp, 16-byte column chunk) for A then B
    constexpr int NA = 16 * CA, NB = 16 * CB;
    constexpr int PER = (NA + NB + 255) / 256;
    auto item = [&](int q, bool &isA, int &kp, int &c8) {
        isA = q < NA;
        const int qq = isA ? q : q - NA;
        const int cc = isA ? CA : CB;
        kp = qq / cc;
        c8 = qq % cc;
    };
    auto load = [&](int k0, uint4 (&rx)[PER][2]) {
#pragma unroll
        for (int p = 0; p < PER; p++) {
            const int q = t + 256 * p;
            rx[p][0] = rx[p][1] = make_uint4(0, 0, 0, 0);
            if (q < NA + NB) {
                bool isA;
                int kp, c8;
                item(q, isA, kp, c8);
                const int col = (isA ? m0 : n0) + 8 * c8;
                const int lim = isA ? M : N;
                const bf16_t *src = isA ? A : B;
                const int ld = isA ? lda : ldb;
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    const int k = k0 + 2 * kp + e;
                    if (k < kend && col < lim) rx[p][e] = *reinterpret_cast<const uint4 *>(src + (int64_t)k * ld + col);
                }
            }
        }
    };
    auto store = [&](int buf, const uint4 (&rx)[PER][2]) {
#pragma unroll
        for (int p = 0; p < PER; p++) {
            const int q = t + 256 * p;
            if (q < NA + NB) {
                bool isA;
                int kp, c8;
                item(q, isA, kp, c8);
                uint4 lo, hi;
                kw_interleave(rx[p][0], rx[p][1], lo, hi);
                unsigned *dst = isA ? &As[buf][kp][8 * c8] : &Bs[buf][kp][8 * c8];
                *reinterpret_cast<uint4 *>(dst) = lo;
                *reinterpret_cast<uint4 *>(dst + 4) = hi;
            }
        }
    };
    f32x16 acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; i++)
#pragma unroll
        for (int j = 0; j < BN; j++) acc[i][j] = f32x16{};
    uint4 rx[PER][2];
    int buf = 0;
    if (kbeg < kend) {
        load(kbeg, rx);
        store(0, rx);
    }
    __syncthreads();
    for (int k0 = kbeg; k0 < kend; k0 += 32) {
        const bool more = k0 + 32 < kend;
        if (more) load(k0 + 32, rx);
#pragma unroll
        for (int kb = 0; kb < 2; kb++) {
            bf16x8 af[BM], bfr[BN];
#pragma unroll
            for (int i = 0; i < BM; i++) {
                const int col = (wm * BM + i) * 32 + r;
                unsigned p[4];
#pragma unroll
                for (int j = 0; j < 4; j++) p[j] = As[buf][8 * kb + 4 * h + j][col];
                af[i] = __builtin_bit_cast(bf16x8, make_uint4(p[0], p[1], p[2], p[3]));
            }
#pragma unroll
            for (int i = 0; i < BN; i++) {
                const int col = (wn * BN + i) * 32 + r;
                unsigned p[4];
#pragma unroll
                for (int j = 0; j < 4; j++) p[j] = Bs[buf][8 * kb + 4 * h + j][col];
                bfr[i] = __builtin_bit_cast(bf16x8, make_uint4(p[0], p[1], p[2], p[3]));
            }
#pragma unroll
            for (int i = 0; i < BM; i++)
#pragma unroll
                for (int j = 0; j < BN; j++) acc[i][j] = mfma32(af[i], bfr[j], acc[i][j]);
        }
        if (more) store(buf ^ 1, rx);
        __syncthreads();
        buf ^= 1;
    }
    // C layout of the 32 x 32 blocks: column = lane % 32 (n), rows 8q + 4h + (0..3) (m)
    float *Cz = C + blockIdx.z * strideC;
#pragma unroll
    for (int i = 0; i < BM; i++)
#pragma unroll
        for (int j = 0; j < BN; j++)
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int m = m0 + (wm * BM + i) * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
                const int n = n0 + (wn * BN + j) * 32 + r;
                if (m < M && n < N) Cz[(int64_t)m * ldc + n] = acc[i][j][v];
            }
}

// dW = dz^T h for the layer shapes of the network: (256, 256) on 128 x 128 tiles, (256, 32)
// (input layer) on 128 x 32 tiles, (16, 256) (output layer) on 32 x 128 tiles.
static int wgrad(const bf16_t *dz, int O, const bf16_t *hp, int I, int n, float *part, int &splits, hipStream_t s)
{
    const int kchunk = ((n + SPLITW - 1) / SPLITW + 31) / 32 * 32;
    splits = (n + kchunk - 1) / kchunk;
    const int64_t stride = (int64_t)O * I;
    if (O % 128 == 0 && I % 128 == 0) {
        hipLaunchKernelGGL((gemm_wgrad_kernel<128, 128, 2>), dim3(I / 128, O / 128, splits), dim3(256), 0, s,
                           dz, O, O, hp, I, I, n, kchunk, part, I, stride);
    } else if (O % 128 == 0 && I == 32) {
        hipLaunchKernelGGL((gemm_wgrad_kernel<128, 32, 4>), dim3(1, O / 128, splits), dim3(256), 0, s,
                           dz, O, O, hp, I, I, n, kchunk, part, I, stride);
    } else if (O <= 32 && O % 8 == 0 && I % 128 == 0) {
        hipLaunchKernelGGL((gemm_wgrad_kernel<32, 128, 1>), dim3(I / 128, 1, splits), dim3(256), 0, s,
                           dz, O, O, hp, I, I, n, kchunk, part, I, stride);
    } else {
        return fail(PROPS_EINVAL, "wgrad: unsupported layer shape %d x %d", O, I);
    }
    PROPS_HIP_TRY(hipGetLastError());
    return PROPS_OK;
}

static int gemm_dh(const GemmArgs &g, hipStream_t s)
{
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, 1);
    hipLaunchKernelGGL(gemm_dh_kernel, grid, dim3(256), 0, s, g);
    PROPS_HIP_TRY(hipGetLastError());
    return PROPS_OK;
}

// One forward + backward pass over rows [row0, row0 + n) of the permuted data; leaves the
// gradient in d->grad and the loss partials (n/256 blocks) in d->lpart.
static int fwd_bwd(props_dnn_s *d, const float *X, const float *Y, int64_t nx, uint64_t pa, uint64_t pc,
                   int64_t row0, int n, hipStream_t s)
{
    int rc;
    FwdArgs a{};
    a.X = X;
    a.nx = nx;
    a.pa = pa;
    a.pc = pc;
    a.row0 = row0;
    a.n = n;
    a.Wf = d->fused;
    a.bias = d->master;
    a.in_lo = d->scal;
    a.in_inv = d->scal + NIN;
    a.h0 = d->h0;
    for (int l = 0; l < 4; l++) {
        a.z[l] = d->zs[l];
        a.h[l] = d->hs[l];
    }
    a.y = d->y;
    if ((rc = launch_fwd(true, a, s))) return rc;
    const int nb = (n + 255) / 256;
    hipLaunchKernelGGL(l1_grad_kernel, dim3(nb), dim3(256), 0, s, d->y, Y, nx, pa, pc, row0, n,
                       d->scal + 2 * NIN, d->scal + 2 * NIN + 2 * NOUT, d->logmask, d->dzo, d->lpart);
    PROPS_HIP_TRY(hipGetLastError());
    // layer by layer, output to input
    const bf16_t *dzl = d->dzo;
    for (int l = NL - 1; l >= 0; l--) {
        const int O = lout(l), I = lin(l);
        const bf16_t *hprev = (l == 0) ? d->h0 : d->hs[l - 1];
        // dW = dz^T h  (M = O, N = I, K = n), split over the batch
        int splits = 0;
        if ((rc = wgrad(dzl, O, hprev, I, n, d->part, splits, s))) return rc;
        const int64_t cnt = (int64_t)O * I;
        hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                           d->part, splits, (int64_t)O * I, cnt, d->grad + kLay::w(l));
        // db = column sums of dz
        const int rows = 256, P = (n + rows - 1) / rows;
        hipLaunchKernelGGL(colsum_partial_kernel, dim3(P), dim3(256), 0, s, dzl, n, O, rows, d->cpart);
        hipLaunchKernelGGL(sum_rows_kernel, dim3((O + 63) / 64), dim3(256), 0, s, d->cpart, P, O, d->grad + kLay::b(l));
        PROPS_HIP_TRY(hipGetLastError());
        if (l > 0) {
            // dz_{l-1} = (dz W) * gelu'(z_{l-1})  (M = n, N = I = 256, K = O)
            bf16_t *out = (dzl == d->dz) ? d->dz2 : d->dz;
            GemmArgs gh{};
            gh.M = n, gh.N = I, gh.K = O;
            gh.A = dzl, gh.lda = O, gh.B = d->nat + kLay::nat(l), gh.ldb = O;
            gh.Cb = out, gh.ldc = I, gh.Z = d->zs[l - 1], gh.ldz = HID;
            if ((rc = gemm_dh(gh, s))) return rc;
            dzl = out;
        }
    }
    return PROPS_OK;
}

static void epoch_perm(uint64_t seed, int epoch, int64_t n, uint64_t &pa, uint64_t &pc)
{
    // the stream starts from the hashed seed (so that neighbouring seeds do not give shifted
    // copies of one stream) xor-ed with an odd multiple of the epoch
    uint64_t st = seed;
    st = splitmix64(st) ^ ((uint64_t)epoch * 0xD1B54A32D192ED03ull);
    // a: an odd multiplier coprime to n; c: any offset
    for (;;) {
        pa = (splitmix64(st) % (uint64_t)n) | 1ull;
        uint64_t x = pa, y = (uint64_t)n;
        while (y) {
            uint64_t r = x % y;
            x = y;
            y = r;
        }
        if (x == 1) break;
    }
    pc = splitmix64(st) % (uint64_t)n;
    if (n == 1) pa = 1, pc = 0;
}

// (h, P, Bilger Z) features of the pressure-based solver's state (Section 4.1), Z Box-Cox
// transformed (Section 4.2): X[0] = h, X[1] = P, X[2] = (Z^lambda - 1) / lambda, X[3..9] = 0.
struct HpzArgs {
    double beta[PROPS_MAX_SPECIES];
    int ns;
    double beta_ox, inv_range, lambda;
    const double *h, *P, *Y;
    double *X;
    int64_t n;
};

__global__ __launch_bounds__(256) void hpz_features_kernel(HpzArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    double b = 0.0;
    for (int i = 0; i < a.ns; i++) b += a.Y[(int64_t)i * a.n + k] * a.beta[i];
    const double Z = fmax((b - a.beta_ox) * a.inv_range, 0.0);
    a.X[k] = a.h[k];
    a.X[a.n + k] = a.P[k];
    a.X[2 * a.n + k] = (pow(Z, a.lambda) - 1.0) / a.lambda;
    for (int f = 3; f < NIN; f++) a.X[(int64_t)f * a.n + k] = 0.0;
}

int dnn_device(const props_dnn_s *d) { return d->device; }

int dnn_eval(props_dnn_s *d, props_mech_s *fb, const props_in *in, const props_out *out, int64_t n,
             int64_t ldy, uint8_t *status, int *fb_idx, int *fb_count, hipStream_t s)
{
    if (!in->P || !in->T || !in->Y) return fail(PROPS_EINVAL, "props_dnn: needs P, T and Y");
    if (d->logmask != kPTYLogMask)
        return fail(PROPS_EINVAL, "props_dnn: the network's log outputs (mask 0x%x) are not those of "
                    "(rho, h, cp, c, mu, lambda); evaluate it with props_dnn_features", d->logmask);
    if (fb && fb->ns != NIN - 2)
        return fail(PROPS_EINVAL, "props_dnn: fallback mechanism has %d species, the network %d", fb->ns, NIN - 2);
    if (fb && (!fb_idx || !fb_count)) return fail(PROPS_EINVAL, "props_dnn: fallback needs index scratch");
    int rc;
    FwdArgs a{};
    a.P = in->P, a.T = in->T, a.Y = in->Y, a.n = n, a.ldy = ldy;
    a.Wf = d->fused, a.bias = d->master;
    a.in_lo = d->scal, a.in_inv = d->scal + NIN;
    a.out_lo = d->scal + 2 * NIN, a.out_rng = d->scal + 2 * NIN + NOUT;
    a.orho = out->rho, a.oh = out->h, a.ocp = out->cp, a.oc = out->c, a.omu = out->mu, a.olam = out->lambda;
    a.status = status;
    if (fb) {
        a.fb_idx = fb_idx;
        a.fb_count = fb_count;
        hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, s, fb_count, 0);
    }
    if ((rc = launch_fwd(false, a, s))) return rc;
    if (fb) {
        props_out po{};
        po.rho = out->rho, po.h = out->h, po.cp = out->cp, po.c = out->c, po.mu = out->mu, po.lambda = out->lambda;
        props_in pi{};
        pi.P = in->P, pi.T = in->T, pi.Y = in->Y;
        rc = launch_pr_indirect(fb, PROPS_PTY, PROPS_MIXED, &pi, &po, n, ldy, fb_idx, fb_count, status,
                                PROPS_ST_OUT_OF_HULL | PROPS_ST_FALLBACK, s);
        if (rc) return rc;
    }
    return PROPS_OK;
}

}  // namespace props

extern "C" {

int props_dnn_create(uint64_t seed, props_dnn_t *out)
{
    if (!out) return fail(PROPS_EINVAL, "props_dnn_create: out is NULL");
    *out = nullptr;
    props_dnn_s *d = new (std::nothrow) props_dnn_s();
    if (!d) return fail(PROPS_ENOMEM, "props_dnn_create: out of host memory");
    if (hipGetDevice(&d->device) != hipSuccess) {
        delete d;
        return fail(PROPS_EHIP, "props_dnn_create: hipGetDevice failed");
    }
    int rc = alloc_dnn(d);
    if (rc) {
        free_dnn(d);
        return rc;
    }
    std::vector<float> h(kLay::total, 0.0f);
    uint64_t st = seed;
    for (int l = 0; l < NL; l++) {
        const double k = 1.0 / std::sqrt((double)tin(l));
        for (int o = 0; o < tout(l); o++)
            for (int i = 0; i < tin(l); i++) h[kLay::w(l) + (size_t)o * lin(l) + i] = (float)((2.0 * u01(st) - 1.0) * k);
        for (int o = 0; o < tout(l); o++) h[kLay::b(l) + o] = (float)((2.0 * u01(st) - 1.0) * k);
    }
    for (int f = 0; f < NIN; f++) d->in_lo[f] = 0.0, d->in_hi[f] = 1.0;
    for (int j = 0; j < NOUT; j++) d->out_lo[j] = 0.0, d->out_hi[j] = 1.0;
    if (hipMemcpy(d->master, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        (rc = upload_scalers(d)) || (rc = refresh_weights(d, nullptr)) ||
        hipDeviceSynchronize() != hipSuccess) {
        free_dnn(d);
        return rc ? rc : fail(PROPS_EHIP, "props_dnn_create: initialisation failed");
    }
    *out = d;
    return PROPS_OK;
}

void props_dnn_destroy(props_dnn_t net)
{
    if (net) free_dnn(net);
}

int props_dnn_get_layer(props_dnn_t d, int l, float *W, float *b)
{
    if (!d || l < 0 || l >= NL) return fail(PROPS_EINVAL, "props_dnn_get_layer: bad network or layer");
    std::vector<float> h((size_t)lout(l) * lin(l) + lout(l));
    PROPS_HIP_TRY(hipMemcpy(h.data(), d->master + kLay::w(l), h.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (int o = 0; o < tout(l); o++) {
        if (W)
            for (int i = 0; i < tin(l); i++) W[(size_t)o * tin(l) + i] = h[(size_t)o * lin(l) + i];
        if (b) b[o] = h[(size_t)lout(l) * lin(l) + o];
    }
    return PROPS_OK;
}

int props_dnn_set_layer(props_dnn_t d, int l, const float *W, const float *b)
{
    if (!d || l < 0 || l >= NL || !W || !b) return fail(PROPS_EINVAL, "props_dnn_set_layer: bad arguments");
    std::vector<float> h((size_t)lout(l) * lin(l) + lout(l), 0.0f);
    for (int o = 0; o < tout(l); o++) {
        for (int i = 0; i < tin(l); i++) h[(size_t)o * lin(l) + i] = W[(size_t)o * tin(l) + i];
        h[(size_t)lout(l) * lin(l) + o] = b[o];
    }
    PROPS_HIP_TRY(hipMemcpy(d->master + kLay::w(l), h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    PROPS_HIP_TRY(hipMemset(d->m + kLay::w(l), 0, h.size() * sizeof(float)));
    PROPS_HIP_TRY(hipMemset(d->v + kLay::w(l), 0, h.size() * sizeof(float)));
    int rc = refresh_weights(d, nullptr);
    if (rc) return rc;
    PROPS_HIP_TRY(hipDeviceSynchronize());
    return PROPS_OK;
}

int props_dnn_get_scalers(props_dnn_t d, double *in_lo, double *in_hi, double *out_lo, double *out_hi)
{
    if (!d) return fail(PROPS_EINVAL, "props_dnn_get_scalers: null network");
    for (int f = 0; f < NIN; f++) {
        if (in_lo) in_lo[f] = d->in_lo[f];
        if (in_hi) in_hi[f] = d->in_hi[f];
    }
    for (int j = 0; j < NOUT; j++) {
        if (out_lo) out_lo[j] = d->out_lo[j];
        if (out_hi) out_hi[j] = d->out_hi[j];
    }
    return PROPS_OK;
}

int props_dnn_set_scalers(props_dnn_t d, const double *in_lo, const double *in_hi, const double *out_lo,
                          const double *out_hi)
{
    if (!d || !in_lo || !in_hi || !out_lo || !out_hi) return fail(PROPS_EINVAL, "props_dnn_set_scalers: null argument");
    for (int f = 0; f < NIN; f++)
        if (!(in_hi[f] >= in_lo[f])) return fail(PROPS_EINVAL, "props_dnn_set_scalers: in_hi < in_lo at %d", f);
    for (int j = 0; j < NOUT; j++)
        if (!(out_hi[j] >= out_lo[j])) return fail(PROPS_EINVAL, "props_dnn_set_scalers: out_hi < out_lo at %d", j);
    std::memcpy(d->in_lo, in_lo, sizeof(d->in_lo));
    std::memcpy(d->in_hi, in_hi, sizeof(d->in_hi));
    std::memcpy(d->out_lo, out_lo, sizeof(d->out_lo));
    std::memcpy(d->out_hi, out_hi, sizeof(d->out_hi));
    return upload_scalers(d);
}

int props_dnn_set_log_outputs(props_dnn_t d, unsigned mask)
{
    if (!d) return fail(PROPS_EINVAL, "props_dnn_set_log_outputs: null network");
    if (mask >> NOUT) return fail(PROPS_EINVAL, "props_dnn_set_log_outputs: mask 0x%x has bits beyond output %d", mask, NOUT - 1);
    d->logmask = mask;
    return PROPS_OK;
}

int props_dnn_get_log_outputs(props_dnn_t d, unsigned *mask)
{
    if (!d || !mask) return fail(PROPS_EINVAL, "props_dnn_get_log_outputs: null argument");
    *mask = d->logmask;
    return PROPS_OK;
}

int props_dnn(props_dnn_t d, props_mech_t fb, const props_in *in, const props_out *out, int64_t n,
              uint8_t *status, void *hip_stream)
{
    ApiRange range_("props_dnn");
    if (!d || !in || !out) return fail(PROPS_EINVAL, "props_dnn: null network, input or output");
    if (n < 0) return fail(PROPS_EINVAL, "props_dnn: n < 0");
    if (n == 0) return PROPS_OK;
    if (n > 0x7fffffffLL) return fail(PROPS_ETOOBIG, "props_dnn: n too large");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc;
    if (fb && n > d->fb_cap) {
        if (d->fb_idx) {
            PROPS_HIP_TRY(hipStreamSynchronize(s));
            (void)hipFree(d->fb_idx);
            d->fb_idx = nullptr;
            d->fb_cap = 0;
        }
        if ((rc = dalloc(&d->fb_idx, (size_t)n))) return rc;
        d->fb_cap = n;
    }
    return dnn_eval(d, fb, in, out, n, n, status, d->fb_idx, d->fb_count, s);
}

int props_dnn_features(props_dnn_t d, const double *X, double *Y, int64_t n, void *hip_stream)
{
    ApiRange range_("props_dnn_features");
    if (!d || !X || !Y) return fail(PROPS_EINVAL, "props_dnn_features: null network, input or output");
    if (n < 0) return fail(PROPS_EINVAL, "props_dnn_features: n < 0");
    if (n == 0) return PROPS_OK;
    if (n > 0x7fffffffLL) return fail(PROPS_ETOOBIG, "props_dnn_features: n too large");
    FwdArgs a{};
    a.Xd = X, a.Yd = Y, a.n = n;
    a.Wf = d->fused, a.bias = d->master;
    a.in_lo = d->scal, a.in_inv = d->scal + NIN;
    a.out_lo = d->scal + 2 * NIN, a.out_rng = d->scal + 2 * NIN + NOUT;
    a.logmask = d->logmask;
    return launch_fwd(false, a, (hipStream_t)hip_stream);
}

int props_features_hpz(const int *atoms, const double *W, int ns, int fuel, int oxidizer, double bc_lambda,
                       const double *h, const double *P, const double *Y, int64_t n, double *X, void *hip_stream)
{
    ApiRange range_("props_features_hpz");
    if (!atoms || !W || !h || !P || !Y || !X) return fail(PROPS_EINVAL, "props_features_hpz: null argument");
    if (ns < 1 || ns > PROPS_MAX_SPECIES) return fail(PROPS_EINVAL, "props_features_hpz: ns = %d", ns);
    if (fuel < 0 || fuel >= ns || oxidizer < 0 || oxidizer >= ns)
        return fail(PROPS_EINVAL, "props_features_hpz: fuel %d / oxidizer %d out of range", fuel, oxidizer);
    if (!(bc_lambda > 0.0 && bc_lambda <= 1.0))
        return fail(PROPS_EINVAL, "props_features_hpz: need 0 < lambda <= 1 (got %g)", bc_lambda);
    double beta[PROPS_MAX_SPECIES];
    for (int i = 0; i < ns; i++) {
        if (!(W[i] > 0.0)) return fail(PROPS_EINVAL, "props_features_hpz: W[%d] <= 0", i);
        beta[i] = (2.0 * atoms[3 * i] + 0.5 * atoms[3 * i + 1] - atoms[3 * i + 2]) / W[i];
    }
    const double beta_fuel = beta[fuel], beta_ox = beta[oxidizer];
    if (!(beta_fuel != beta_ox))
        return fail(PROPS_EINVAL, "props_features_hpz: fuel and oxidizer have the same coupling function");
    if (n < 0) return fail(PROPS_EINVAL, "props_features_hpz: n < 0");
    if (n == 0) return PROPS_OK;
    HpzArgs a{};
    for (int i = 0; i < ns; i++) a.beta[i] = beta[i];
    a.ns = ns;
    a.beta_ox = beta_ox;
    a.inv_range = 1.0 / (beta_fuel - beta_ox);
    a.lambda = bc_lambda;
    a.h = h, a.P = P, a.Y = Y, a.X = X, a.n = n;
    // a dispatch holds at most 2^32 - 1 work-items: n <= 2^32 - 256
    if (n > 0x100000000LL - 256) return fail(PROPS_ETOOBIG, "props_features_hpz: n too large");
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(hpz_features_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, a);
    PROPS_HIP_TRY(hipGetLastError());
    return PROPS_OK;
}

static int fit_scalers_dev(props_dnn_s *d, const float *X, const float *Y, int64_t n, hipStream_t s)
{
    const int B = 256;
    const int64_t per = (n + B - 1) / B;
    double *part = nullptr;
    int rc;
    if ((rc = dalloc(&part, (size_t)B * 2 * (NIN + NOUT)))) return rc;
    hipLaunchKernelGGL(minmax_partial_kernel, dim3(B, NIN), dim3(256), 0, s, X, n, NIN, 0u, per, part);
    hipLaunchKernelGGL(minmax_partial_kernel, dim3(B, NOUT), dim3(256), 0, s, Y, n, NOUT, d->logmask, per,
                       part + (size_t)B * 2 * NIN);
    std::vector<double> h((size_t)B * 2 * (NIN + NOUT));
    hipError_t e = hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(part);
    if (e != hipSuccess) return fail(PROPS_EHIP, "fit scalers: %s", hipGetErrorString(e));
    for (int f = 0; f < NIN + NOUT; f++) {
        double lo = INFINITY, hi = -INFINITY;
        for (int b = 0; b < B; b++) {
            lo = std::min(lo, h[((size_t)f * B + b) * 2]);
            hi = std::max(hi, h[((size_t)f * B + b) * 2 + 1]);
        }
        if (!std::isfinite(lo) || !std::isfinite(hi)) return fail(PROPS_EINVAL, "train_dnn: non-finite data in column %d", f);
        if (f < NIN) d->in_lo[f] = lo, d->in_hi[f] = hi;
        else d->out_lo[f - NIN] = lo, d->out_hi[f - NIN] = hi;
    }
    return upload_scalers(d);
}

int props_dnn_grad(props_dnn_t d, const float *X, const float *Y, int64_t n, float *grad, float *loss,
                   void *hip_stream)
{
    ApiRange range_("props_dnn_grad");
    if (!d || !X || !Y || !grad) return fail(PROPS_EINVAL, "props_dnn_grad: null argument");
    if (n < 1 || n > MAX_BATCH) return fail(PROPS_EINVAL, "props_dnn_grad: need 1 <= n <= %d", MAX_BATCH);
    hipStream_t s = (hipStream_t)hip_stream;
    int rc;
    if ((rc = ensure_train_scratch(d))) return rc;
    if ((rc = fwd_bwd(d, X, Y, n, 1, 0, 0, (int)n, s))) return rc;
    std::vector<float> g(kLay::total), lp((n + 255) / 256);
    PROPS_HIP_TRY(hipMemcpyAsync(g.data(), d->grad, g.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    PROPS_HIP_TRY(hipMemcpyAsync(lp.data(), d->lpart, lp.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    PROPS_HIP_TRY(hipStreamSynchronize(s));
    size_t o = 0;
    for (int l = 0; l < NL; l++) {
        for (int r = 0; r < tout(l); r++)
            for (int i = 0; i < tin(l); i++) grad[o++] = g[kLay::w(l) + (size_t)r * lin(l) + i];
        for (int r = 0; r < tout(l); r++) grad[o++] = g[kLay::b(l) + r];
    }
    if (loss) {
        double sl = 0;
        for (float v : lp) sl += v;
        *loss = (float)(sl / ((double)n * NOUT));
    }
    return PROPS_OK;
}

int train_dnn(props_dnn_t d, const float *X, const float *Y, int64_t n, const props_train_cfg *cfg,
              props_train_report *rep, void *hip_stream)
{
    ApiRange range_("train_dnn");
    if (!d || !X || !Y || !cfg) return fail(PROPS_EINVAL, "train_dnn: null argument");
    if (n < 1) return fail(PROPS_EINVAL, "train_dnn: n < 1");
    const int batch = cfg->batch ? cfg->batch : MAX_BATCH;
    if (batch < 256 || batch > MAX_BATCH || batch % 256) return fail(PROPS_EINVAL, "train_dnn: batch must be a multiple of 256 in [256, %d]", MAX_BATCH);
    if (cfg->epochs < 0 || !(cfg->lr > 0)) return fail(PROPS_EINVAL, "train_dnn: bad epochs or learning rate");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc;
    auto t0 = std::chrono::steady_clock::now();
    if ((rc = ensure_train_scratch(d))) return rc;
    if (cfg->fit_scalers && (rc = fit_scalers_dev(d, X, Y, n, s))) return rc;
    const int total = cfg->total_epochs > 0 ? cfg->total_epochs : std::max(1, d->epoch + cfg->epochs);
    const float b1 = cfg->beta1 > 0 ? cfg->beta1 : 0.9f, b2 = cfg->beta2 > 0 ? cfg->beta2 : 0.999f;
    const float eps = cfg->eps > 0 ? cfg->eps : 1e-8f;
    const int64_t steps_per_epoch = (n + batch - 1) / batch;
    const int64_t P = (int64_t)kLay::total;
    std::vector<float> lp;
    int64_t steps = 0;
    float *lsum = nullptr;   // per-step loss partial sums of one epoch
    const int lblocks = batch / 256;
    if ((rc = dalloc(&lsum, (size_t)steps_per_epoch * lblocks))) return rc;
    for (int e = 0; e < cfg->epochs; e++) {
        uint64_t pa, pc;
        epoch_perm(cfg->seed, d->epoch, n, pa, pc);
        const double prog = std::min(1.0, (double)d->epoch / total);
        hipLaunchKernelGGL(fill_float_kernel, dim3((unsigned)((steps_per_epoch * lblocks + 255) / 256)), dim3(256), 0, s,
                           lsum, steps_per_epoch * lblocks, 0.0f);
        const float lr = (float)(cfg->lr_min + 0.5 * (cfg->lr - cfg->lr_min) * (1.0 + std::cos(M_PI * prog)));
        for (int64_t st = 0; st < steps_per_epoch; st++) {
            const int64_t row0 = st * batch;
            const int m = (int)std::min<int64_t>(batch, n - row0);
            if ((rc = fwd_bwd(d, X, Y, n, pa, pc, row0, m, s))) {
                (void)hipFree(lsum);
                return rc;
            }
            PROPS_HIP_TRY(hipMemcpyAsync(lsum + st * lblocks, d->lpart, sizeof(float) * ((m + 255) / 256),
                                         hipMemcpyDeviceToDevice, s));
            d->step++;
            const float bc1 = 1.0f - std::pow(b1, (float)d->step), bc2 = 1.0f - std::pow(b2, (float)d->step);
            hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, d->master, d->grad,
                               d->m, d->v, P, lr, b1, b2, eps, bc1, bc2);
            if ((rc = refresh_weights(d, s))) {
                (void)hipFree(lsum);
                return rc;
            }
            steps++;
        }
        lp.resize((size_t)steps_per_epoch * lblocks);
        hipError_t err = hipMemcpyAsync(lp.data(), lsum, lp.size() * sizeof(float), hipMemcpyDeviceToHost, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        if (err != hipSuccess) {
            (void)hipFree(lsum);
            return fail(PROPS_EHIP, "train_dnn: %s", hipGetErrorString(err));
        }
        double sl = 0;
        for (float v : lp) sl += v;
        if (rep && rep->loss) rep->loss[e] = (float)(sl / ((double)n * NOUT));
        d->epoch++;
    }
    (void)hipFree(lsum);
    PROPS_HIP_TRY(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) {
        rep->epochs_run = cfg->epochs;
        rep->steps = steps;
        rep->seconds = secs;
        rep->samples_per_s = secs > 0 ? (double)n * cfg->epochs / secs : 0.0;
    }
    return PROPS_OK;
}

// ---- checkpoint: "PROPSDNN" v2 | step | epoch | log-output mask | scalers | master | m | v
// (v1, without the mask, loads with the (P, T, Y) surrogate's mask)
int props_dnn_save(props_dnn_t d, const char *path)
{
    ApiRange range_("props_dnn_save");
    if (!d || !path) return fail(PROPS_EINVAL, "props_dnn_save: null argument");
    const size_t P = kLay::total;
    std::vector<float> buf(3 * P);
    PROPS_HIP_TRY(hipDeviceSynchronize());
    PROPS_HIP_TRY(hipMemcpy(buf.data(), d->master, P * 4, hipMemcpyDeviceToHost));
    PROPS_HIP_TRY(hipMemcpy(buf.data() + P, d->m, P * 4, hipMemcpyDeviceToHost));
    PROPS_HIP_TRY(hipMemcpy(buf.data() + 2 * P, d->v, P * 4, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(PROPS_EINVAL, "props_dnn_save: cannot open %s", path);
    const char magic[8] = {'P', 'R', 'O', 'P', 'S', 'D', 'N', 'N'};
    const uint32_t ver = 2;
    const uint64_t np = P;
    const uint32_t mask = d->logmask;
    bool ok = std::fwrite(magic, 8, 1, f) == 1 && std::fwrite(&ver, 4, 1, f) == 1 && std::fwrite(&np, 8, 1, f) == 1 &&
              std::fwrite(&d->step, 8, 1, f) == 1 && std::fwrite(&d->epoch, 4, 1, f) == 1 &&
              std::fwrite(&mask, 4, 1, f) == 1 &&
              std::fwrite(d->in_lo, sizeof(d->in_lo), 1, f) == 1 && std::fwrite(d->in_hi, sizeof(d->in_hi), 1, f) == 1 &&
              std::fwrite(d->out_lo, sizeof(d->out_lo), 1, f) == 1 && std::fwrite(d->out_hi, sizeof(d->out_hi), 1, f) == 1 &&
              std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? PROPS_OK : fail(PROPS_EINVAL, "props_dnn_save: write to %s failed", path);
}

int props_dnn_load(const char *path, props_dnn_t *out)
{
    ApiRange range_("props_dnn_load");
    if (!path || !out) return fail(PROPS_EINVAL, "props_dnn_load: null argument");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(PROPS_EINVAL, "props_dnn_load: cannot open %s", path);
    char magic[8];
    uint32_t ver = 0;
    uint64_t np = 0;
    props_dnn_t d = nullptr;
    int rc = props_dnn_create(0, &d);
    if (rc) {
        std::fclose(f);
        return rc;
    }
    const size_t P = kLay::total;
    std::vector<float> buf(3 * P);
    uint32_t mask = kPTYLogMask;
    bool ok = std::fread(magic, 8, 1, f) == 1 && std::memcmp(magic, "PROPSDNN", 8) == 0 && std::fread(&ver, 4, 1, f) == 1 &&
              (ver == 1 || ver == 2) && std::fread(&np, 8, 1, f) == 1 && np == P && std::fread(&d->step, 8, 1, f) == 1 &&
              std::fread(&d->epoch, 4, 1, f) == 1 && (ver == 1 || std::fread(&mask, 4, 1, f) == 1) &&
              (mask >> NOUT) == 0 && std::fread(d->in_lo, sizeof(d->in_lo), 1, f) == 1 &&
              std::fread(d->in_hi, sizeof(d->in_hi), 1, f) == 1 && std::fread(d->out_lo, sizeof(d->out_lo), 1, f) == 1 &&
              std::fread(d->out_hi, sizeof(d->out_hi), 1, f) == 1 && std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) {
        props_dnn_destroy(d);
        return fail(PROPS_EINVAL, "props_dnn_load: %s is not a valid checkpoint", path);
    }
    d->logmask = mask;
    if (hipMemcpy(d->master, buf.data(), P * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->m, buf.data() + P, P * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->v, buf.data() + 2 * P, P * 4, hipMemcpyHostToDevice) != hipSuccess ||
        (rc = upload_scalers(d)) || (rc = refresh_weights(d, nullptr)) || hipDeviceSynchronize() != hipSuccess) {
        props_dnn_destroy(d);
        return rc ? rc : fail(PROPS_EHIP, "props_dnn_load: upload failed");
    }
    *out = d;
    return PROPS_OK;
}

}  // extern "C"
