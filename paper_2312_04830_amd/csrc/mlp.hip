// MLP surrogate of the property path (paper, Section 4): BF16 matrix-core kernels.
//
// Network: NIN inputs -> nh hidden layers of 256 (GELU) -> nout outputs, L1 loss; nh is 3
// (the paper's networks, Section 4.1) or 4, nout is 1..6.
//
// Inference / training forward: one fused kernel.  Cells are the N dimension of
// v_mfma_f32_32x32x16_bf16 (32 cells per wave) and features the M and K dimensions: the
// 32x32 FP32 accumulator of a 32-feature output block holds, in each lane, 16 features of
// one cell, which are exactly the 2 x 8 bf16 values that lane contributes to two K blocks
// of the next layer's B operand.  Activations therefore never leave registers; the next
// layer's weights are stored with the matching permutation of their input index.  The bias
// rides on the matrix cores as well: each weight row carries the FP32 bias split into three
// bf16 parts (hi + mid + lo, exact), which one extra K block multiplies by a constant
// (1, 1, 1, 0, ...) operand, so the accumulator starts from zero and no vector instruction
// touches the bias.  GELU (tanh form, hardware exp2 and reciprocal) is applied in FP32 on
// the accumulators, then packed to bf16 with v_cvt_pk_bf16_f32 (round to nearest even).
//
// Weight streaming: one persistent 8-wave workgroup per CU (two waves per SIMD) walks 256-cell
// tiles; every tile walks the same sequence of weight blocks (the hidden layers' 32-row output
// blocks, the output layer, then the next tile's layer 0), staged a pair of blocks at a time
// with global_load_lds into a ring of three slot pairs in LDS (101 KB), two pairs ahead of the
// one in use, so staging overlaps the matrix-core work.
//
// Backward: dz of every hidden layer in one fused pass (mlp_bwd_kernel: per tile, dz of a layer
// is (dz of the next) x W with the GELU derivative at the saved bf16 z, kept in registers from
// layer to layer like the forward's activations, the transposed weights streamed through the
// same kind of ring); dW = dz^T h on the 32x32x16 MFMA with both operands k-major, split over
// the batch with a fixed-order reduction (training is deterministic and resumable bit for
// bit), the bias gradient as dz^T times ones in the same pass; Adam on FP32 master weights.
// The forward keeps bf16 copies of pre-activations and activations for the backward, and
// writes the output layer's L1 gradient directly.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "props_internal.hpp"
#include "trace.hpp"

namespace props {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned short bf16_t;  // storage type of a bfloat16

constexpr int NIN = PROPS_DNN_IN, NOUT = PROPS_DNN_OUT, HID = PROPS_DNN_HIDDEN;
constexpr int MIN_HIDDEN = 3, MAX_HIDDEN = 4;
constexpr int IN_PAD = 32;     // input columns of the layer-0 weights and of saved inputs
constexpr int OUT_PAD = 16;    // output rows of the last layer's weights and output gradients
constexpr int HROW = HID + 8;  // bf16 per fused row of a 256-input layer: inputs, bias hi/mid/lo, 5 zeros
constexpr int FK0 = 16;        // layer-0 K in the fused layout: one 16-deep K block
constexpr int IROW = FK0 + 8;  // bf16 per layer-0 fused row (48 B): 16 inputs, bias hi/mid/lo, 5 zeros
constexpr int FOUT_ROWS = 32;  // last layer padded to one 32-row output block
constexpr int FWD_WAVES = 8;                              // one workgroup per CU, 2 waves per SIMD
constexpr int FWD_THREADS = FWD_WAVES * 64;
constexpr int CELLS_PER_WAVE = 32;
constexpr int TILE_CELLS = FWD_WAVES * CELLS_PER_WAVE;   // 256
constexpr int SLOT_BYTES = 32 * HROW * 2;                 // one 32-row block: 16,896 B
constexpr int NRING = 3;                                  // ring of three slot pairs
constexpr int LDS_BYTES = NRING * 2 * SLOT_BYTES;         // 101,376 B per workgroup
constexpr int L0_BYTES = HID * IROW * 2;                  // layer 0 whole: 12,288 B, one slot
static_assert(L0_BYTES <= SLOT_BYTES, "layer 0 fits one slot");
constexpr int MAX_BATCH = 65536;
// floats per training sample row: the inputs, the targets, padding to 64 bytes
constexpr int SAMPLE_FLOATS = 16;
static_assert(NIN + NOUT <= SAMPLE_FLOATS, "a sample row holds the inputs and the targets");
// Batch splits of the weight-gradient GEMMs (multiples of 8) and the prefetch depth of their
// loaders, in 32-cell steps.  Fewer splits write and reduce fewer FP32 partials but give each
// workgroup a longer serial walk; on a 65,536 batch the three 256 x 256 layers in one launch
// take 63 us with 64 splits each (768 workgroups of 32 steps) and training runs 2.5 % faster
// with 32, 7 % slower with 128; 128 splits of the input and output layers take 13-14 us each.
constexpr int SPLIT_HID = 32;
constexpr int SPLIT_IO = 128;
constexpr int WG_DEPTH = 4;

// LDS fragment prefetch distance of the A-fragment stream, in matrix-core steps
constexpr int FPF = 3;
// Outputs of the (P, T, Y) surrogate trained on their logarithm: rho, cp, mu, lambda
// (bits 0, 2, 4, 5; h and c cross or approach zero and stay linear).
constexpr unsigned kPTYLogMask = 0x35u;

// ------------------------------------------------------------------ layout
// Weight layers 0..nh: layer 0 maps the inputs to 256 features, layers 1..nh-1 are 256 x 256,
// layer nh is the output layer.  Padded (out, in) of each layer in the FP32 master vector
// (W row-major then b), and its offsets there, in the transposed natural bf16 copy and in the
// fused bf16 layout.
__host__ __device__ inline int lout(int l, int nh) { return l == 0 ? HID : (l == nh ? OUT_PAD : HID); }
__host__ __device__ inline int lin(int l) { return l == 0 ? IN_PAD : HID; }
__host__ __device__ inline int lrow(int l) { return l == 0 ? IROW : HROW; }
__host__ __device__ inline size_t w_off(int l)
{
    return l == 0 ? 0 : (size_t)IN_PAD * HID + HID + (size_t)(l - 1) * (HID * HID + HID);
}
__host__ __device__ inline size_t b_off(int l, int nh) { return w_off(l) + (size_t)lout(l, nh) * lin(l); }
__host__ __device__ inline size_t total_params(int nh) { return w_off(nh) + (size_t)OUT_PAD * HID + OUT_PAD; }
static_assert((IN_PAD * HID + HID) % 4 == 0 && (HID * HID + HID) % 4 == 0 && (OUT_PAD * HID + OUT_PAD) % 4 == 0,
              "layer parameter counts are multiples of four (the step kernel takes four parameters a thread)");
// split-K partials of one step, every layer side by side (W then b of each split, as in the
// master)
inline size_t part_floats(int nh)
{
    return (size_t)SPLIT_IO * ((size_t)HID * IN_PAD + HID + (size_t)OUT_PAD * HID + OUT_PAD) +
           (size_t)(nh - 1) * SPLIT_HID * ((size_t)HID * HID + HID);
}
__host__ __device__ inline size_t f_off(int l) { return l == 0 ? 0 : (size_t)HID * IROW + (size_t)(l - 1) * HID * HROW; }
__host__ __device__ inline size_t f_total(int nh) { return f_off(nh) + (size_t)FOUT_ROWS * HROW; }
// Backward-data layout: the transposed weights of layers 1..nh, rows = the layer's inputs
// (256 hidden features), K = the layer's outputs.  Hidden layers l = 1..nh-1 take the
// accumulator permutation on K (their dz arrives in registers) and rows of HROW; the output
// layer (K = 16, dz read from memory in natural order) takes rows of IROW, after them.
__host__ __device__ inline size_t bf_off(int l, int nh) { return l < nh ? (size_t)(l - 1) * HID * HROW : (size_t)(nh - 1) * HID * HROW; }
__host__ __device__ inline size_t bf_total(int nh) { return (size_t)(nh - 1) * HID * HROW + (size_t)HID * IROW; }
// Layout of the saved hidden-layer arrays (z, h, and dz written over z; logically
// [n][256]): the four features 32 ob + 8 q + 4 hh + (0..3) of a cell sit next to those of the
// other lanes of the same wave that hold them, 64 lanes x 8 bytes = 512 bytes per (32-cell
// group, block ob, q), in lane order (hh, cell % 32).  Every save by the forward and every
// reload by the backward (the same lane mapping) is then one coalesced 512-byte access, and
// cells 2c, 2c + 1 of a group with the same four features are 16 contiguous bytes, which the
// weight-gradient loader turns into (k even, k odd) pairs.
__host__ __device__ inline int64_t tm_idx(int64_t cell, int f)
{
    return ((((cell >> 5) * 8 + (f >> 5)) * 4 + ((f >> 3) & 3)) * 64 + ((f >> 2) & 1) * 32 + (cell & 31)) * 4 + (f & 3);
}
// true (unpadded) shapes
__host__ __device__ inline int tout(int l, int nh, int nout) { return l == nh ? nout : HID; }
__host__ __device__ inline int tin(int l) { return l == 0 ? NIN : HID; }

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
// gelu_f in two halves, the same operations in the same order: the exponential, then the rest
__device__ __forceinline__ float gelu_exp_f(float x) { return __builtin_amdgcn_exp2f(x * __builtin_fmaf(kG1, x * x, kG0)); }
__device__ __forceinline__ float gelu_fin_f(float x, float e) { return x * __builtin_amdgcn_rcpf(1.0f + e); }

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
    // inference inputs (SoA doubles, species rows ldy apart) ...
    const double *P, *T, *Y;
    int64_t ldy;
    // ... or the training set, one 64-byte sample per row ([nx][16] float: the 10 inputs, the
    // raw targets, zeros), read in the order of the epoch permutation
    const float *XY;
    int64_t nx;
    uint64_t pa, pc;
    int64_t row0;        // first permuted row of this batch
    int64_t n;           // cells (rows) this launch covers
    int nhid, nout;      // hidden layers, outputs
    const bf16_t *Wf;    // fused-layout weights (with the bias parts) of all layers
    const double *in_lo, *in_inv;   // [10] input box
    const double *out_lo, *out_rng, *out_inv; // [6] target box
    unsigned logmask;               // bit j: output j was trained on its logarithm
    // ... or inference on raw feature-major inputs [10][n], outputs [nout][n]
    const double *Xd;
    double *Yd;
    // inference outputs
    double *orho, *oh, *ocp, *oc, *omu, *olam;
    uint8_t *status;
    int *fb_idx, *fb_count;         // fallback list (cells outside the box / non-physical)
    // training: saves for the backward and the output layer's L1 gradient
    bf16_t *h0;                     // [n][32] scaled inputs
    bf16_t *zs, *hs;                // pre-activations and activations of hidden layer l:
    int64_t lstride;                // [n][256] each, at zs + l lstride and hs + l lstride
    bf16_t *dzo;                    // [n][16] d loss / d output
    float *lpart;                   // [tiles * FWD_WAVES] sums of |y - t| per wave
};

// Issue global_load_lds of `bytes` (a multiple of 16) from src to the LDS slot dst: each
// lane's 16 bytes go straight to LDS, without passing through registers; one 1 KB chunk per
// wave and instruction.  Completion is awaited by the caller (vmcnt, then a barrier).
__device__ __forceinline__ void stage_async(unsigned char *dst, const bf16_t *src, int bytes)
{
    // chunk addresses are wave-uniform (scalar base + this lane's 16-byte offset), and the lane
    // offset is formed here, at each call, not hoisted out of the tile loop into registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned lo = (threadIdx.x & 63) * 16u;
    asm volatile("" : "+v"(lo));
    const unsigned char *s = reinterpret_cast<const unsigned char *>(src);
    constexpr int PER_WAVE = (SLOT_BYTES / 1024 + FWD_WAVES) / FWD_WAVES;   // 1 KB chunks per wave (5)
#pragma unroll
    for (int r = 0; r < PER_WAVE; r++) {
        const int c = wave + FWD_WAVES * r;
        if (c * 1024 + (int)lo < bytes)
            __builtin_amdgcn_global_load_lds((const void *)(s + c * 1024 + lo),
                                             (__attribute__((address_space(3))) void *)(dst + c * 1024), 16, 0, 0);
    }
}

// Weights of block k of the per-tile sequence: 0 .. 8 (nh - 1) - 1 the 32-row output blocks of
// the hidden 256 x 256 layers in order, 8 (nh - 1) the output layer, 8 (nh - 1) + 1 layer 0
// (whole) of the next tile.
__device__ __forceinline__ void step_weights(const FwdArgs &a, int k, const bf16_t *&src, int &bytes)
{
    const int nh = a.nhid;
    if (k == 8 * (nh - 1) + 1) {
        src = a.Wf;
        bytes = L0_BYTES;
    } else if (k == 8 * (nh - 1)) {
        src = a.Wf + f_off(nh);
        bytes = SLOT_BYTES;
    } else {
        const int l = 1 + k / 8, ob = k % 8;
        src = a.Wf + f_off(l) + (size_t)ob * 32 * HROW;
        bytes = SLOT_BYTES;
    }
}

// Fill the two slots of ring pair `rp` (0..2) with the weights of sequence pair p: blocks 2p
// and 2p + 1.  The weight base goes through an empty asm so that the per-lane load addresses are
// formed here, at each call: hoisted out of the tile loop (they do not depend on the tile) they
// would occupy a hundred VGPR pairs.
__device__ __forceinline__ void stage_pair(unsigned char *lds, const FwdArgs &a, int rp, int p)
{
    FwdArgs b = a;
    const bf16_t *wf = a.Wf;
    asm volatile("" : "+s"(wf));
    b.Wf = wf;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const bf16_t *src;
        int bytes;
        step_weights(b, 2 * p + j, src, bytes);
        stage_async(lds + (2 * rp + j) * SLOT_BYTES, src, bytes);
    }
}

// Wait for every outstanding memory operation of this wave, then meet the workgroup's other
// waves.  The barrier carries no memory fence (the full wait already orders this wave's
// accesses; the empty asm statements keep the compiler from moving any across): with the
// fences of __syncthreads the inference forward is register-allocated worse (58 VGPRs
// spilled, against none).
__device__ __forceinline__ void wait_then_barrier()
{
    __builtin_amdgcn_s_waitcnt(0);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Start of the pair held in ring pair rp.  On entry the pair's weights are in LDS for every
// wave (certified at the previous pair's start).  Here this wave's loads of the next pair
// (issued at the previous pair's start) land, the barrier makes that true of every wave and
// tells that every wave is done with the previous pair, whose ring pair then receives the
// weights of sequence pair pn (two pairs ahead).  The A-fragment stream may thus read the
// next pair's slots at any time during this pair.
__device__ __forceinline__ void pair_top(unsigned char *lds, const FwdArgs &a, int rp, int pn, bool stage)
{
    wait_then_barrier();
    if (stage) stage_pair(lds, a, rp == 0 ? NRING - 1 : rp - 1, pn);
}

// Per-lane LDS byte addresses of one block's A fragments: `k` the weight K blocks (row col,
// K slot 8h), `b` the bias parts (row col, K slot past the inputs; for lane half 1 the B
// operand is zero there).  Formed through an empty asm at each block, so that the compiler
// does not hoist one pair per block and slot out of the tile loop.
struct BlkAddr {
    unsigned k, b;
};
__device__ __forceinline__ BlkAddr hid_addr(unsigned slot_off, int col, int h)
{
    unsigned k = slot_off + (unsigned)(col * HROW + 8 * h) * 2u;
    unsigned b = slot_off + (unsigned)(col * HROW + HID) * 2u;
    asm volatile("" : "+v"(k), "+v"(b));
    return {k, b};
}
__device__ __forceinline__ BlkAddr l0_addr(unsigned slot_off, int col, int h)
{
    unsigned k = slot_off + (unsigned)(col * IROW + 8 * h) * 2u;
    unsigned b = slot_off + (unsigned)(col * IROW + FK0) * 2u;
    asm volatile("" : "+v"(k), "+v"(b));
    return {k, b};
}
__device__ __forceinline__ bf16x8 lds_at(const unsigned char *lds, unsigned addr, int off)
{
    return *reinterpret_cast<const bf16x8 *>(lds + addr + off);
}
// A fragment of step s of a 256-input block: s = 0 the bias parts, s >= 1 K block s - 1
__device__ __forceinline__ bf16x8 hid_frag(const unsigned char *lds, BlkAddr ad, int s)
{
    return s == 0 ? lds_at(lds, ad.b, 0) : lds_at(lds, ad.k, (s - 1) * 32);
}
// A fragment of step s of layer 0: sub-block s / 2, its bias parts (s even) or inputs (s odd)
__device__ __forceinline__ bf16x8 l0_frag(const unsigned char *lds, BlkAddr ad, int s)
{
    const int off = (s >> 1) * 32 * IROW * 2;
    return (s & 1) ? lds_at(lds, ad.k, off) : lds_at(lds, ad.b, off);
}

// The A-fragment stream: FPF fragments in flight ahead of the matrix-core step that uses them,
// continuing across block and pair boundaries.
struct Ring {
    bf16x8 f[FPF];
};
__device__ __forceinline__ bf16x8 ring_step(Ring &r, bf16x8 incoming)
{
    const bf16x8 c = r.f[0];
#pragma unroll
    for (int d = 0; d + 1 < FPF; d++) r.f[d] = r.f[d + 1];
    r.f[FPF - 1] = incoming;
    return c;
}

// Training saves of one 32-feature block of a hidden layer: bf16 pre-activations z into zl and
// the packed bf16 activations p (8 pairs) into hl, in the saved-array layout (tm_idx).  The
// stores are non-temporal: the saves are read back only by later kernels, and kept out of
// the cache they leave room there for the weights that every tile re-stages.
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void save_block(bf16_t *zl, bf16_t *hl, int64_t cell, int ob, int h, const f32x16 &z,
                                           const unsigned *p)
{
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int64_t off = tm_idx(cell, 32 * ob + 8 * q + 4 * h);
        const u32x2 zv = {pack_bf16x2(z[4 * q], z[4 * q + 1]), pack_bf16x2(z[4 * q + 2], z[4 * q + 3])};
        const u32x2 hv = {p[2 * q], p[2 * q + 1]};
        __builtin_nontemporal_store(zv, reinterpret_cast<u32x2 *>(zl + off));
        __builtin_nontemporal_store(hv, reinterpret_cast<u32x2 *>(hl + off));
    }
}

// GELU of the 16 accumulator values of one block, packed into the two bf16x8 B-operand
// fragments of the next layer.
__device__ __forceinline__ void gelu_block(const f32x16 &z, bf16x8 &lo, bf16x8 &hi, unsigned *p)
{
#pragma unroll
    for (int q = 0; q < 8; q++) p[q] = pack_bf16x2(gelu_f(z[2 * q]), gelu_f(z[2 * q + 1]));
    lo = __builtin_bit_cast(bf16x8, make_uint4(p[0], p[1], p[2], p[3]));
    hi = __builtin_bit_cast(bf16x8, make_uint4(p[4], p[5], p[6], p[7]));
}

// Layer 0: 16 matrix-core steps, the bias and input MFMAs of each 32-row sub-block ob, with
// the GELU of sub-block ob - 1 beside them.  Fills act[0..13] (and, with `save`, writes the
// training saves of sub-blocks 0..6); returns sub-block 7's accumulator, whose GELU is pending.
// The stream continues into the first 256-input block at `nx`.
__device__ __forceinline__ f32x16 l0_block(const unsigned char *lds, BlkAddr cur, BlkAddr nx, Ring &ring,
                                           bf16x8 x0, bf16x8 (&act)[16], bf16x8 ones, const FwdArgs &a,
                                           int64_t cell, bool save)
{
    const int h = (threadIdx.x & 63) >> 5;
    constexpr int NS = 16;
    f32x16 zp = {};
#pragma unroll
    for (int ob = 0; ob < 8; ob++) {
        f32x16 z;
#pragma unroll
        for (int t = 0; t < 2; t++) {
            const int s = 2 * ob + t, u = s + FPF;
            const bf16x8 af = ring_step(ring, u < NS ? l0_frag(lds, cur, u) : hid_frag(lds, nx, u - NS));
            z = (t == 0) ? mfma32(af, ones, f32x16{}) : mfma32(af, x0, z);
        }
        if (ob > 0) {
            unsigned p[8];
            gelu_block(zp, act[2 * ob - 2], act[2 * ob - 1], p);
            if (save) save_block(a.zs, a.hs, cell, ob - 1, h, zp, p);
        }
        zp = z;
        __builtin_amdgcn_sched_barrier(0);
    }
    return zp;
}

// One 32-row output block of a 256-input layer at `cur`: returns bias + W act in 17
// matrix-core steps (the bias block, then K blocks 0..15), while the GELU of the pending
// block's accumulator pz is formed one value per step into the packed bf16 pairs pg.  Each
// step is a scheduling region of its own (the LDS read FPF steps ahead, one MFMA, the first
// part of one or two GELU values and the rest of the previous step's), so that the vector
// work of a step runs in the shadow of its MFMA.  The stream continues into the next block
// at `nx`, a 256-input block or (NEXT_L0) the next tile's layer 0.  FIRST: pz is the previous
// layer's last block, i.e. act[14], act[15]; its 16 values are started by step 14 (two at
// step 0) and finished a step later, act[14] (values 0..7) is filled before step 15 and
// act[15] (values 8..15) before step 16, the steps that read them.
template <bool FIRST, bool NEXT_L0>
__device__ __forceinline__ f32x16 hid_block(const unsigned char *lds, BlkAddr cur, BlkAddr nx, Ring &ring,
                                            bf16x8 (&act)[16], const f32x16 &pz, unsigned (&pg)[8], bf16x8 ones)
{
    constexpr int NS = 17;
    f32x16 acc = {};
    float ex[16], gv[16];
    // values whose GELU starts at step s (FIRST: two at step 0, one at steps 1..14; else one
    // at steps 0..15); each is finished one step later
    const auto v0 = [](int s) { return FIRST ? (s == 0 ? 0 : s + 1) : s; };
    const auto nv = [](int s) { return FIRST ? (s == 0 ? 2 : (s < 15 ? 1 : 0)) : (s < 16 ? 1 : 0); };
#pragma unroll
    for (int s = 0; s < NS; s++) {
        if (FIRST && s == 15) act[14] = __builtin_bit_cast(bf16x8, make_uint4(pg[0], pg[1], pg[2], pg[3]));
        if (FIRST && s == 16) act[15] = __builtin_bit_cast(bf16x8, make_uint4(pg[4], pg[5], pg[6], pg[7]));
        const int u = s + FPF;
        const bf16x8 af = ring_step(ring, u < NS ? hid_frag(lds, cur, u)
                                                 : (NEXT_L0 ? l0_frag(lds, nx, u - NS) : hid_frag(lds, nx, u - NS)));
        acc = (s == 0) ? mfma32(af, ones, f32x16{}) : mfma32(af, act[s - 1], acc);
        // Each part of a GELU is pinned to its step: the activations are needed only by the
        // next layer, and without the pin the compiler sinks the GELUs of whole blocks out of
        // the matrix-core steps into one run of vector work.  The chain of one value (seven
        // dependent operations) is split over two steps: this step's exponentials, then the
        // rest of the previous step's values.
#pragma unroll
        for (int w = 0; w < nv(s); w++) {
            const int v = v0(s) + w;
            ex[v] = gelu_exp_f(pz[v]);
            asm volatile("" : "+v"(ex[v]));
        }
        if (s > 0) {
#pragma unroll
            for (int w = 0; w < nv(s - 1); w++) {
                const int v = v0(s - 1) + w;
                gv[v] = gelu_fin_f(pz[v], ex[v]);
                asm volatile("" : "+v"(gv[v]));
                if (v & 1) pg[v >> 1] = pack_bf16x2(gv[v - 1], gv[v]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    return acc;
}

// Raw inputs of one cell for this lane (inference: doubles; training: the float features of
// the permuted sample), loaded a block ahead of their use.
template <bool TRAIN>
struct RawIn {
    typedef typename std::conditional<TRAIN, float, double>::type T;
    T x[NIN];
};

// Issue the loads of one tile's inputs for this lane's cell (`cell` < n) or, in training,
// of its permuted sample `sidx`.
template <bool TRAIN>
__device__ __forceinline__ void load_inputs(const FwdArgs &a, int64_t cell, int64_t sidx, RawIn<TRAIN> &r)
{
    if (TRAIN) {
        // a permuted sample is one 64-byte row: its inputs are three 16-byte loads
        const float4 *p = reinterpret_cast<const float4 *>(a.XY + SAMPLE_FLOATS * sidx);
        const float4 v0 = p[0], v1 = p[1], v2 = p[2];
        r.x[0] = v0.x, r.x[1] = v0.y, r.x[2] = v0.z, r.x[3] = v0.w;
        r.x[4] = v1.x, r.x[5] = v1.y, r.x[6] = v1.z, r.x[7] = v1.w;
        r.x[8] = v2.x, r.x[9] = v2.y;
    } else if (a.Xd) {
#pragma unroll
        for (int f = 0; f < NIN; f++) r.x[f] = a.Xd[(int64_t)f * a.n + cell];
    } else {
        r.x[0] = a.P[cell];
        r.x[1] = a.T[cell];
#pragma unroll
        for (int f = 0; f < NIN - 2; f++) r.x[2 + f] = a.Y[(int64_t)f * a.ldy + cell];
    }
}

// Training targets of this lane's output rows 4h + r (r = 0..3; at most 6 outputs, so rows
// 8 and up of the block carry none) for sample sidx
__device__ __forceinline__ void load_targets(const FwdArgs &a, int64_t sidx, int h, float (&t)[4])
{
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int j = 4 * h + r;
        t[r] = j < a.nout ? a.XY[SAMPLE_FLOATS * sidx + NIN + j] : 0.0f;
    }
}

// Scaled bf16 B operand of layer 0 from the raw inputs (half 0: features 0..7, half 1: 8, 9),
// and in inference the hull / sanity flag of the cell; training saves the scaled inputs.
template <bool TRAIN>
__device__ __forceinline__ bf16x8 scale_inputs(const FwdArgs &a, const RawIn<TRAIN> &r, bool live, int64_t cell,
                                               int h, uint8_t &flag)
{
    float xs[8];
#pragma unroll
    for (int j = 0; j < 8; j++) xs[j] = 0.0f;
    flag = 0;
    if (live) {
        double raw[NIN];
#pragma unroll
        for (int f = 0; f < NIN; f++) raw[f] = (double)r.x[f];
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
                // a feature constant in the training data (in_inv = 0) scales to 0 for the
                // network, but the box still holds only that one value
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
    if (TRAIN && live) {
        // saved inputs keep IN_PAD columns; 16..31 stay zero from allocation
        *reinterpret_cast<uint4 *>(a.h0 + cell * IN_PAD + 8 * h) = *reinterpret_cast<uint4 *>(p);
    }
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<uint4 *>(p));
}

// Fused forward of the surrogate: per 256-cell tile, layer 0, the hidden 256 x 256 layers and
// the output layer, with activations in registers (cells are the N side of
// v_mfma_f32_32x32x16_bf16, 32 per wave) and the weights streamed through LDS one 32-row block
// at a time.  The per-tile sequence of blocks (the hidden layers' 8 blocks each, the output
// layer, then layer 0 of the next tile) is staged in pairs by LDS DMA into a ring of three slot
// pairs, two pairs ahead; one barrier per pair.  The next tile's inputs are loaded at the start
// of the output pair and used after its matrix-core work; the outputs are written before the
// next tile's layer 0, a whole block ahead of the next wait on memory.
template <bool TRAIN>
__global__ __launch_bounds__(FWD_THREADS, 1) void mlp_fwd_kernel(FwdArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5;         // lane half: K slots 8h..8h+7 (A, B); rows 8q + 4h.. (C)
    const int col = lane & 31;       // cell within the wave's 32-cell block (B, C); A row
    const int nh = a.nhid;
    const int PT = 1 + 4 * (nh - 1);        // pairs per tile: (2 + 8 (nh - 1)) blocks
    const int64_t ntiles = (a.n + TILE_CELLS - 1) / TILE_CELLS;
    if ((int64_t)blockIdx.x >= ntiles) return;   // whole workgroup: no barrier is skipped by part of it
    // B operand of the bias block: K slots 0..2 are 1 (they meet the bias hi, mid, lo parts of
    // each weight row), every other slot 0
    bf16x8 ones = bf16x8{};
    if (h == 0) ones = __builtin_bit_cast(bf16x8, make_uint4(0x3f803f80u, 0x00003f80u, 0u, 0u));
    // Training blocks write their bf16 pre-activations and activations; the inference build
    // carries no save code.
    constexpr bool saves = TRAIN;
    constexpr unsigned PAIR = 2 * SLOT_BYTES;
    const auto next_rp = [](int r) { return r == NRING - 1 ? 0 : r + 1; };

    // prologue: layer 0 of the first tile into slot 1 of ring pair 2, the tile's pairs 0 and 1
    // into ring pairs 0 and 1; the first tile's inputs; the first fragments of layer 0
    {
        const bf16_t *wf = a.Wf;
        asm volatile("" : "+s"(wf));
        stage_async(lds + (2 * 2 + 1) * SLOT_BYTES, wf, L0_BYTES);
    }
    stage_pair(lds, a, 0, 0);
    stage_pair(lds, a, 1, 1);
    int64_t cell = (int64_t)blockIdx.x * TILE_CELLS + wave * CELLS_PER_WAVE + col;
    bool live = cell < a.n;
    int64_t sidx = TRAIN ? perm_index(a.row0 + (live ? cell : 0), a.pa, a.pc, a.nx) : 0;
    uint8_t flag;
    bf16x8 x0;                       // B operand of layer 0: the scaled inputs
    {
        RawIn<TRAIN> r;
        load_inputs<TRAIN>(a, live ? cell : 0, sidx, r);
        x0 = scale_inputs<TRAIN>(a, r, live, cell, h, flag);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int rp = 2;                      // ring pair of the current pair
    Ring ring;
    {
        const BlkAddr l0 = l0_addr(2 * PAIR + SLOT_BYTES, col, h);
#pragma unroll
        for (int d = 0; d < FPF; d++) ring.f[d] = l0_frag(lds, l0, d);
    }

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const bool more = tile + gridDim.x < ntiles;
        bf16x8 act[16];              // B operand of a 256-input layer: one bf16x8 per 16-deep K block
        bf16x8 nxt[14];              // the layer's outputs of blocks 0..6 as they are formed
        f32x16 pz;                   // accumulator of the block whose GELU is pending

        // ---- layer 0: slot 1 of the current pair; the GELU of its blocks 0..6 gives
        // act[0..13], that of block 7 is left pending
        pz = l0_block(lds, l0_addr(rp * PAIR + SLOT_BYTES, col, h), hid_addr(next_rp(rp) * PAIR, col, h), ring, x0,
                      act, ones, a, cell, saves && live);

        // ---- hidden 256 x 256 layers: one 32-row output block per step, whose matrix-core work
        // is interleaved with the GELU of the block before it; at block 0 that is the previous
        // layer's last block, whose two K blocks of act are needed only by the last two steps.
        // Sequence block k = 8 (l - 1) + ob; even ob open a pair (slot 0), odd ob are slot 1.
#pragma unroll 1
        for (int l = 1; l < nh; l++) {
            bf16_t *zprev = nullptr, *hprev = nullptr, *zcur = nullptr, *hcur = nullptr;
            if (saves) {
                zcur = a.zs + l * a.lstride, hcur = a.hs + l * a.lstride;
                zprev = zcur - a.lstride, hprev = hcur - a.lstride;
            }
#pragma unroll
            for (int ob = 0; ob < 8; ob++) {
                if (!(ob & 1)) {
                    rp = next_rp(rp);
                    const int pn = 4 * (l - 1) + ob / 2 + 2;   // sequence pair two ahead
                    pair_top(lds, a, rp, pn < PT ? pn : pn - PT, pn < PT || more);
                }
                const unsigned base = rp * PAIR;
                const BlkAddr cur = hid_addr((ob & 1) ? base + SLOT_BYTES : base, col, h);
                const BlkAddr nx = hid_addr((ob & 1) ? next_rp(rp) * PAIR : base + SLOT_BYTES, col, h);
                unsigned pg[8];
                f32x16 acc;
                if (ob == 0) {
                    acc = hid_block<true, false>(lds, cur, nx, ring, act, pz, pg, ones);
                    if (saves && live) save_block(zprev, hprev, cell, 7, h, pz, pg);
                } else {
                    acc = hid_block<false, false>(lds, cur, nx, ring, act, pz, pg, ones);
                    const int pb = ob - 1;
                    nxt[2 * pb] = __builtin_bit_cast(bf16x8, make_uint4(pg[0], pg[1], pg[2], pg[3]));
                    nxt[2 * pb + 1] = __builtin_bit_cast(bf16x8, make_uint4(pg[4], pg[5], pg[6], pg[7]));
                    if (saves && live) save_block(zcur, hcur, cell, pb, h, pz, pg);
                }
                pz = acc;
            }
#pragma unroll
            for (int kb = 0; kb < 14; kb++) act[kb] = nxt[kb];
        }

        // ---- output layer (linear): slot 0 of the last pair of the tile, whose slot 1 holds
        // the next tile's layer 0; its matrix-core work is interleaved with the GELU of the last
        // hidden layer's last block.  The next tile's inputs (and in training this tile's
        // targets) are loaded meanwhile.
        rp = next_rp(rp);
        pair_top(lds, a, rp, 1, more);
        const int64_t ncell = cell + (int64_t)gridDim.x * TILE_CELLS;
        const bool nlive = more && ncell < a.n;
        const int64_t nsidx = (TRAIN && more) ? perm_index(a.row0 + (nlive ? ncell : 0), a.pa, a.pc, a.nx) : 0;
        RawIn<TRAIN> rn;
        if (more) load_inputs<TRAIN>(a, nlive ? ncell : 0, nsidx, rn);
        float tg[4];
        if (TRAIN) load_targets(a, sidx, h, tg);
        {
            unsigned pg[8];
            const f32x16 acc = hid_block<true, true>(lds, hid_addr(rp * PAIR, col, h),
                                                     l0_addr(rp * PAIR + SLOT_BYTES, col, h), ring, act, pz, pg, ones);
            if (saves && live)
                save_block(a.zs + (nh - 1) * a.lstride, a.hs + (nh - 1) * a.lstride, cell, 7, h, pz, pg);
            uint8_t nflag = 0;
            bf16x8 nx0 = x0;
            if (more) nx0 = scale_inputs<TRAIN>(a, rn, nlive, ncell, h, nflag);
            if (TRAIN) {
                // L1 loss on the scaled targets: rows 8q + 4h + r (q = 0, 1) of the block are
                // outputs j; d loss / d y_j = sign(y_j - t_j) / (rows * nout)
                const float scale = 1.0f / ((float)a.n * (float)a.nout);
                float lsum = 0.f;
                float dv[8];
#pragma unroll
                for (int q = 0; q < 2; q++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int j = 8 * q + 4 * h + r;
                        float d = 0.f;
                        if (live && q == 0 && j < a.nout) {
                            double tr = (double)tg[r];
                            if (a.logmask >> j & 1u) tr = log(tr);
                            const float t = (float)((tr - a.out_lo[j]) * a.out_inv[j]);
                            const float diff = acc[4 * q + r] - t;
                            lsum += fabsf(diff);
                            d = (diff > 0.f) ? scale : ((diff < 0.f) ? -scale : 0.f);
                        }
                        dv[4 * q + r] = d;
                    }
                if (live) {
#pragma unroll
                    for (int q = 0; q < 2; q++)
                        *reinterpret_cast<uint2 *>(a.dzo + cell * OUT_PAD + 8 * q + 4 * h) =
                            make_uint2(pack_bf16x2(dv[4 * q], dv[4 * q + 1]), pack_bf16x2(dv[4 * q + 2], dv[4 * q + 3]));
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
                if (lane == 0) a.lpart[tile * FWD_WAVES + wave] = lsum;
            } else {
                if (live) {
                    // rows 4h + v, v = 0..3, are outputs j (half 0: 0..3, half 1: 4, 5), back to
                    // target units; those trained on their logarithm through exp, as 2^(y log2 e)
                    // in single precision (the network's own precision)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int j = 4 * h + v;
                        if (j < a.nout) {
                            double y = __builtin_fma((double)acc[v], a.out_rng[j], a.out_lo[j]);
                            if (a.logmask >> j & 1u)
                                y = (double)__builtin_amdgcn_exp2f((float)(y * 1.4426950408889634));
                            double *dst = a.Yd ? a.Yd + (int64_t)j * a.n
                                               : (j == 0 ? a.orho : j == 1 ? a.oh : j == 2 ? a.ocp
                                                  : j == 3 ? a.oc : j == 4 ? a.omu : a.olam);
                            if (dst) dst[cell] = y;
                        }
                    }
                }
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
            x0 = nx0;
            flag = nflag;
        }
        cell = ncell;
        live = nlive;
        sidx = nsidx;
    }
    __builtin_amdgcn_s_waitcnt(0);   // no weight load still in flight when the workgroup ends
}

// ------------------------------------------------------------------ fused backward (data)
// dz of every hidden layer for a 256-cell tile in one pass, output layer to input:
//   dz_{nh-1} = (W_out^T dz_out) o GELU'(z_{nh-1}),  dz_{t-1} = (W_t^T dz_t) o GELU'(z_{t-1}),
// with the same layout tricks as the forward: cells are the N side of the MFMA (32 per wave),
// the transposed weights (rows = the layer's inputs, K = its outputs in the accumulator
// permutation) stream through the ring of three LDS slot pairs, and each dz stays in
// registers as the next layer's B operand.  Each dz_t is written over z_t (the lane that
// reads a z value is the one that writes its dz, two blocks later), where the weight-gradient
// GEMMs read it.  W_out^T (K = 16) sits in its own LDS region after the ring.
struct BwdArgs {
    const bf16_t *Wb;      // backward-data weights (bf_off layout)
    const bf16_t *dzo;     // [n][16] d loss / d output
    bf16_t *zs;            // hidden layer t's z at zs + t lstride, overwritten by its dz
    int64_t lstride;
    int64_t n;
    int nhid;
};
constexpr int BWD_WOUT = NRING * 2 * SLOT_BYTES;          // byte offset of W_out^T in LDS
constexpr int BWD_LDS_BYTES = BWD_WOUT + HID * IROW * 2;  // 113,664 B

// weights of block k of the per-tile backward sequence: hidden layer l = nh - 1 - k / 8,
// 32-row block k % 8 of its transpose
__device__ __forceinline__ void bwd_stage_pair(unsigned char *lds, const BwdArgs &a, int rp, int p)
{
    const bf16_t *wb = a.Wb;
    asm volatile("" : "+s"(wb));
    const int nh = a.nhid;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int k = 2 * p + j;
        const int l = nh - 1 - k / 8, ob = k % 8;
        stage_async(lds + (2 * rp + j) * SLOT_BYTES, wb + bf_off(l, nh) + (size_t)ob * 32 * HROW, SLOT_BYTES);
    }
}

__device__ __forceinline__ void bwd_pair_top(unsigned char *lds, const BwdArgs &a, int rp, int pn, bool stage)
{
    wait_then_barrier();
    if (stage) bwd_stage_pair(lds, a, rp == 0 ? NRING - 1 : rp - 1, pn);
}

// The 16 z values of one block of hidden layer t for this lane (rows 32 ob + 8q + 4h + r),
// four 8-byte loads from the saved-array layout (tm_idx), and the matching dz store
struct ZBlk {
    uint2 q[4];
};
__device__ __forceinline__ void load_zblk(const bf16_t *zl, int64_t cell, int ob, int h, ZBlk &z)
{
#pragma unroll
    for (int q = 0; q < 4; q++) z.q[q] = *reinterpret_cast<const uint2 *>(zl + tm_idx(cell, 32 * ob + 8 * q + 4 * h));
}
__device__ __forceinline__ float zval(const ZBlk &z, int v)
{
    const uint2 w = z.q[v >> 2];
    const unsigned u = ((v & 3) < 2) ? w.x : w.y;
    return (v & 1) ? __builtin_bit_cast(float, u & 0xffff0000u) : __builtin_bit_cast(float, u << 16);
}
__device__ __forceinline__ void store_dzblk(bf16_t *zl, int64_t cell, int ob, int h, const unsigned (&pg)[8])
{
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const u32x2 v = {pg[2 * q], pg[2 * q + 1]};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x2 *>(zl + tm_idx(cell, 32 * ob + 8 * q + 4 * h)));
    }
}

// One 32-row block of a hidden layer's transpose (16 K blocks, no bias) at `cur`, with the
// pending block's dz = dh o GELU'(z) formed one value per step into pg (the forward's
// interleave, with GELU' in place of GELU).  FIRST: the pending block is the previous
// layer's last one (act[14], act[15]): its 16 values are done by step 13 (two at steps 0
// and 1) and act[14], act[15] are filled before steps 14 and 15, which read them.  The
// stream continues into the block at `nx`.
template <bool FIRST>
__device__ __forceinline__ f32x16 bwd_block(const unsigned char *lds, BlkAddr cur, BlkAddr nx, Ring &ring,
                                            bf16x8 (&act)[16], const f32x16 &pz, const ZBlk &zp, unsigned (&pg)[8])
{
    constexpr int NS = 16;
    f32x16 acc = {};
    float gv[16];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        if (FIRST && s == 14) {
            act[14] = __builtin_bit_cast(bf16x8, make_uint4(pg[0], pg[1], pg[2], pg[3]));
            act[15] = __builtin_bit_cast(bf16x8, make_uint4(pg[4], pg[5], pg[6], pg[7]));
        }
        const int u = s + FPF;
        const bf16x8 af = ring_step(ring, u < NS ? lds_at(lds, cur.k, u * 32) : lds_at(lds, nx.k, (u - NS) * 32));
        acc = (s == 0) ? mfma32(af, act[0], f32x16{}) : mfma32(af, act[s], acc);
        // FIRST: two values at steps 0 and 1, one at steps 2..13 (all 16 before step 14)
        const int v0 = FIRST ? (s < 2 ? 2 * s : s + 2) : s;
        const int nv = FIRST ? (s < 2 ? 2 : (s < 14 ? 1 : 0)) : 1;
#pragma unroll
        for (int w = 0; w < nv; w++) {
            const int v = v0 + w;
            gv[v] = pz[v] * gelu_grad_f(zval(zp, v));
            if (v & 1) pg[v >> 1] = pack_bf16x2(gv[v - 1], gv[v]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    return acc;
}

__device__ __forceinline__ void dz_epilogue(const f32x16 &pz, const ZBlk &zp, unsigned (&pg)[8])
{
#pragma unroll
    for (int q = 0; q < 8; q++)
        pg[q] = pack_bf16x2(pz[2 * q] * gelu_grad_f(zval(zp, 2 * q)), pz[2 * q + 1] * gelu_grad_f(zval(zp, 2 * q + 1)));
}

__global__ __launch_bounds__(FWD_THREADS, 1) void mlp_bwd_kernel(BwdArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5;
    const int col = lane & 31;
    const int nh = a.nhid;
    const int PT = 4 * (nh - 1);            // pairs per tile: 8 (nh - 1) hidden blocks
    const int64_t ntiles = (a.n + TILE_CELLS - 1) / TILE_CELLS;
    if ((int64_t)blockIdx.x >= ntiles) return;
    constexpr unsigned PAIR = 2 * SLOT_BYTES;
    const auto next_rp = [](int r) { return r == NRING - 1 ? 0 : r + 1; };

    // prologue: W_out^T into its region, the first two pairs into ring pairs 0 and 1
    {
        const bf16_t *wb = a.Wb;
        asm volatile("" : "+s"(wb));
        stage_async(lds + BWD_WOUT, wb + bf_off(nh, nh), HID * IROW * 2);
    }
    bwd_stage_pair(lds, a, 0, 0);
    bwd_stage_pair(lds, a, 1, 1);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int rp = 2;                              // the ring pair before the first hidden pair
    Ring ring;
    {
        const BlkAddr b0 = hid_addr(0, col, h);
#pragma unroll
        for (int d = 0; d < FPF; d++) ring.f[d] = lds_at(lds, b0.k, d * 32);
    }

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const bool more = tile + gridDim.x < ntiles;
        const int64_t cell = tile * TILE_CELLS + wave * CELLS_PER_WAVE + col;
        const bool live = cell < a.n;
        const int64_t cl = live ? cell : 0;  // dead lanes read cell 0 and write nothing
        bf16x8 act[16];
        bf16x8 nxt[14];
        f32x16 pz;
        // The tile's blocks j = 8 (nh - 1 - t) + ob run from hidden layer t = nh - 1 (the
        // output step) down to t = 0.  z of block j is loaded two blocks ahead, into a
        // three-deep shift register: zq[0] the pending block's, zq[1] the current one's,
        // zq[2] the next one's.
        const auto zrow = [&](int t) { return a.zs + t * a.lstride; };
        ZBlk zq[3];
        const auto zshift = [&](int t2, int ob2) {   // after a block: turn, then load block (t2, ob2)
            zq[0] = zq[1];
            zq[1] = zq[2];
            if (t2 >= 0) load_zblk(zrow(t2), cl, ob2, h, zq[2]);
        };
        load_zblk(zrow(nh - 1), cl, 0, h, zq[1]);
        load_zblk(zrow(nh - 1), cl, 1, h, zq[2]);
        // ---- output layer: dh_{nh-1} = W_out^T dz_out, eight 32-row blocks of one MFMA each;
        // the dz of block ob - 1 is formed beside block ob
        const bf16x8 dzb = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(a.dzo + cl * OUT_PAD + 8 * h));
        {
            const unsigned wl = l0_addr((unsigned)BWD_WOUT, col, h).k;   // row 32 ob + col, K slot 8h
#pragma unroll
            for (int ob = 0; ob < 8; ob++) {
                const bf16x8 af = lds_at(lds, wl, ob * 32 * IROW * 2);
                const f32x16 z = mfma32(af, dzb, f32x16{});
                if (ob > 0) {
                    unsigned pg[8];
                    dz_epilogue(pz, zq[0], pg);
                    act[2 * ob - 2] = __builtin_bit_cast(bf16x8, make_uint4(pg[0], pg[1], pg[2], pg[3]));
                    act[2 * ob - 1] = __builtin_bit_cast(bf16x8, make_uint4(pg[4], pg[5], pg[6], pg[7]));
                    if (live) store_dzblk(zrow(nh - 1), cl, ob - 1, h, pg);
                }
                pz = z;
                // block j + 2 = ob + 2: still the output step's, or layer nh - 2's first two
                if (ob + 2 < 8) zshift(nh - 1, ob + 2);
                else zshift(nh - 2, ob - 6);
                __builtin_amdgcn_sched_barrier(0);
            }
        }

        // ---- hidden layers l = nh - 1 .. 1 (weights W_l): dh_{l-1} = W_l^T dz_l, then
        // dz_{l-1} = dh o GELU'(z_{l-1}); ring sequence block k = 8 (nh - 1 - l) + ob, even
        // ob open a pair
#pragma unroll 1
        for (int l = nh - 1; l >= 1; l--) {
            const int t = l - 1;             // the hidden layer whose dz this pass forms
#pragma unroll
            for (int ob = 0; ob < 8; ob++) {
                const int kseq = 8 * (nh - 1 - l) + ob;
                if (!(ob & 1)) {
                    rp = next_rp(rp);
                    const int pn = kseq / 2 + 2;
                    bwd_pair_top(lds, a, rp, pn < PT ? pn : pn - PT, pn < PT || more);
                }
                const unsigned base = rp * PAIR;
                const BlkAddr cur = hid_addr((ob & 1) ? base + SLOT_BYTES : base, col, h);
                const BlkAddr nx = hid_addr((ob & 1) ? next_rp(rp) * PAIR : base + SLOT_BYTES, col, h);
                unsigned pg[8];
                f32x16 acc;
                if (ob == 0) {
                    // pending: the last block of layer t + 1
                    acc = bwd_block<true>(lds, cur, nx, ring, act, pz, zq[0], pg);
                    if (live) store_dzblk(zrow(t + 1), cl, 7, h, pg);
                } else {
                    acc = bwd_block<false>(lds, cur, nx, ring, act, pz, zq[0], pg);
                    nxt[2 * ob - 2] = __builtin_bit_cast(bf16x8, make_uint4(pg[0], pg[1], pg[2], pg[3]));
                    nxt[2 * ob - 1] = __builtin_bit_cast(bf16x8, make_uint4(pg[4], pg[5], pg[6], pg[7]));
                    if (live) store_dzblk(zrow(t), cl, ob - 1, h, pg);
                }
                pz = acc;
                if (ob + 2 < 8) zshift(t, ob + 2);
                else zshift(t - 1, ob - 6);     // none past layer 0 (t - 1 < 0)
            }
#pragma unroll
            for (int kb = 0; kb < 14; kb++) act[kb] = nxt[kb];
        }
        // ---- the tile's last block (layer 0, block 7): its dz has no MFMA beside it
        {
            unsigned pg[8];
            dz_epilogue(pz, zq[0], pg);
            if (live) store_dzblk(zrow(0), cl, 7, h, pg);
        }
        // the next tile's first hidden pair is the next ring pair; its fragments were
        // prefetched by this tile's last hidden block
    }
    __builtin_amdgcn_s_waitcnt(0);
}

// ------------------------------------------------------------------ training helpers
// Where each layer's split-K partials sit: layer l's split z holds its W and b (in master
// order) at part[l] + z * (off[l + 1] - off[l]); off[l] = w_off(l).
struct GradParts {
    int64_t off[MAX_HIDDEN + 2];
    const float *part[MAX_HIDDEN + 1];
    int splits[MAX_HIDDEN + 1];
    int nl;
};

// bf16 copies of one master weight (element i of layer l, rows x cols) in the forward's fused
// layout and, after layer 0, the backward-data layout
__device__ __forceinline__ void put_weight(bf16_t *fused, bf16_t *bwd, int l, int nh, int64_t i, float wv)
{
    const int cols = lin(l), rowlen = lrow(l);
    const int o = (int)(i / cols), c = (int)(i % cols);
    const bf16_t b = to_bf16(wv);
    if (l >= 1) {
        // backward-data layout: row c, K slot of output o
        const int brow = (l == nh) ? IROW : HROW;
        bwd[bf_off(l, nh) + (int64_t)c * brow + ((l == nh) ? o : kslot(o))] = b;
    }
    // layer 0 keeps the natural input order in its one 16-deep K block (inputs >= 16 are
    // padding); later layers take the permutation of the accumulator layout
    if (l == 0 && c >= FK0) return;
    fused[f_off(l) + (int64_t)o * rowlen + ((l == 0) ? c : kslot(c))] = b;
}

// a bias in the fused layout: three bf16 parts hi + mid + lo after the row's inputs (exact:
// each part takes the next 8 bits of the FP32 significand)
__device__ __forceinline__ void put_bias(bf16_t *fused, int l, int o, float bv)
{
    const bf16_t hi = to_bf16(bv);
    const float r1 = bv - bf16_to_f(hi);
    const bf16_t mid = to_bf16(r1);
    const bf16_t lo = to_bf16(r1 - bf16_to_f(mid));
    bf16_t *dst = fused + f_off(l) + (int64_t)o * lrow(l) + (l == 0 ? FK0 : HID);
    dst[0] = hi;
    dst[1] = mid;
    dst[2] = lo;
}

// Four lanes per four master parameters e .. e + 3 (layer sizes and offsets are multiples of
// four): lane r of the group sums the splits z = r, r + 4, r + 8, ... in order (16-byte
// loads, sixteen in flight), and the four lane sums are added as (s0 + s1) + (s2 + s3), the
// same expression in every lane of the group, so the gradient g = sum_z part_z[e] is one
// fixed-order, deterministic split-K reduction.  Then lane r takes parameter e + r.  Without
// Adam, g is written to grad.  With Adam: the moments and the FP32 master take the step
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,  w -= lr (m / bc1) / (sqrt(v / bc2) + eps)
// (bc1, bc2: the bias corrections 1 - b^t), and the new weight goes straight to its bf16 copies.
// One lane per four parameters, summing every split, took 23 us per training step (about
// 800 waves on the 1024 SIMDs, each with a long serial chain of loads).
constexpr int GS_VEC = 4, GS_BATCH = 16, GS_THREADS = 256, GS_LANES = 4;
typedef float gs_vec_t __attribute__((ext_vector_type(GS_VEC)));
__global__ __launch_bounds__(GS_THREADS) void grad_step_kernel(GradParts L, int nh, float *grad, float *w, float *m,
                                                        float *v, bf16_t *fused, bf16_t *bwd, int adam, float lr,
                                                        float b1, float b2, float eps, float bc1, float bc2)
{
    constexpr int VEC = GS_VEC, NB = GS_BATCH, R = GS_LANES;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = (int)(tid % R);
    const int64_t e0 = VEC * (tid / R);
    if (e0 >= L.off[L.nl]) return;   // whole groups of R lanes leave together
    int l = 0;
    while (l + 1 < L.nl && e0 >= L.off[l + 1]) l++;
    const int64_t i0 = e0 - L.off[l], cnt = L.off[l + 1] - L.off[l];
    const gs_vec_t *src = reinterpret_cast<const gs_vec_t *>(L.part[l] + i0);
    const int64_t zs = cnt / VEC;
    const int S = L.splits[l];
    float g[VEC] = {};
    int z = r;
    for (; z + R * (NB - 1) < S; z += R * NB) {   // NB partials in flight, summed in order
        gs_vec_t pv[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) pv[j] = __builtin_nontemporal_load(src + (z + R * j) * zs);
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
            for (int u = 0; u < VEC; u++) g[u] += pv[j][u];
    }
    for (; z < S; z += R) {
        const gs_vec_t pv = __builtin_nontemporal_load(src + z * zs);
#pragma unroll
        for (int u = 0; u < VEC; u++) g[u] += pv[u];
    }
    // (s0 + s1) + (s2 + s3) in every lane: the xor-1 partner's sum first, then the xor-2
    // partner's pair sum (addition commutes exactly, so the four lanes agree bit for bit)
    static_assert(R == 4, "the butterfly below adds four lanes");
#pragma unroll
    for (int u = 0; u < VEC; u++) {
        g[u] += __shfl_xor(g[u], 1);
        g[u] += __shfl_xor(g[u], 2);
    }
    const float gr = r == 0 ? g[0] : r == 1 ? g[1] : r == 2 ? g[2] : g[3];
    const int64_t e = e0 + r, i = i0 + r;
    if (!adam) {
        grad[e] = gr;
        return;
    }
    const int64_t nwt = (int64_t)lout(l, nh) * lin(l);
    const float mi = b1 * m[e] + (1.f - b1) * gr;
    const float vi = b2 * v[e] + (1.f - b2) * gr * gr;
    m[e] = mi;
    v[e] = vi;
    const float wn = w[e] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[e] = wn;
    if (i < nwt) put_weight(fused, bwd, l, nh, i, wn);
    else put_bias(fused, l, (int)(i - nwt), wn);
}

// FP32 master -> its bf16 copies (the forward's fused layout with the biases, the
// backward-data layout), all layers
__global__ void convert_weights_kernel(const float *master, bf16_t *fused, bf16_t *bwd, int nh)
{
    const int l = blockIdx.y;
    const int rows = lout(l, nh);
    const int64_t cnt = (int64_t)rows * lin(l);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x)
        put_weight(fused, bwd, l, nh, e, master[w_off(l) + e]);
    for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < rows; o += gridDim.x * blockDim.x)
        put_bias(fused, l, o, master[b_off(l, nh) + o]);
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

namespace props {

// Weight gradient C_z[m][n] = sum_{k in split z} A[k][m] B[k][n], with both operands stored
// k-major ([batch][feature] activations and output gradients), on v_mfma_f32_32x32x16_bf16,
// K in steps of 32.  The matrix cores want each lane's eight bf16 consecutive along K, so tiles
// are staged in LDS as bf16 pairs (k even, k odd), four pairs (k .. k + 7) side by side per
// column: a fragment is then one 16-byte LDS read straight into the operand's registers.
// Double-buffered in LDS, one barrier per step.
// A tile of TM x TN outputs per workgroup of 4 waves arranged WAVES_M x (4 / WAVES_M), each
// wave BM x BN blocks of 32 x 32.  Columns at or beyond M (N) are loaded from the operand's
// first columns and not written (a column of A only reaches row m of C), so the 16-row output
// layer runs on a 32-row tile.  The workgroups of the first column tile also sum the A columns
// over their K range (Cb: the bias gradient's partials, the column sums of dz) on the matrix
// cores, as A^T times a ones operand, in the same fixed order on every run.
// LDS rows of (W + 1) columns x 4 dwords: 4 banks apart modulo 64, so that the 8-byte writes of
// a wave's row-pair x column-group items and the 16-byte fragment reads meet no bank twice
constexpr int KW_PAD = 1;
// bf16 pairs from two dwords, one v_perm_b32 each: low halves (lo.lo, hi.lo) and high halves
// (lo.hi, hi.hi)
__device__ __forceinline__ unsigned pair_lo(unsigned lo, unsigned hi) { return __builtin_amdgcn_perm(hi, lo, 0x05040100u); }
__device__ __forceinline__ unsigned pair_hi(unsigned lo, unsigned hi) { return __builtin_amdgcn_perm(hi, lo, 0x07060302u); }

__device__ __forceinline__ void kw_interleave(uint4 x, uint4 y, uint4 &lo, uint4 &hi)
{
    // x: row 2kp, y: row 2kp + 1, eight bf16 columns each -> eight (x_j, y_j) pairs
    lo = make_uint4(pair_lo(x.x, y.x), pair_hi(x.x, y.x), pair_lo(x.y, y.y), pair_hi(x.y, y.y));
    hi = make_uint4(pair_lo(x.z, y.z), pair_hi(x.z, y.z), pair_lo(x.w, y.w), pair_hi(x.w, y.w));
}

// (cells 2kp, 2kp + 1) x four features, as one 16-byte load from the saved-array layout
// (tm_idx): {c f0 f1, c f2 f3, c+1 f0 f1, c+1 f2 f3} -> the four (c, c+1) pairs
__device__ __forceinline__ uint4 kw_interleave4(uint4 x)
{
    return make_uint4(pair_lo(x.x, x.z), pair_hi(x.x, x.z), pair_lo(x.y, x.w), pair_hi(x.y, x.w));
}

// One operand of the weight-gradient GEMM: W (TM or TN) columns starting at c0, K rows.  SAVED:
// the saved-array layout (tm_idx, 256 features); otherwise row-major [K][ld].  A work item is
// one row pair rp (K rows 4 rp .. 4 rp + 3 of the step) times a column group: four features
// (two 16-byte pieces of the saved layout, 32 contiguous bytes: cells 4 rp .. 4 rp + 1 and
// 4 rp + 2 .. 4 rp + 3) or eight columns (four 16-byte row loads).  Items run along the
// operand's contiguous direction, so consecutive lanes read consecutive memory.
template <int W, bool SAVED>
struct WgOperand {
    static constexpr int CG = SAVED ? W / 4 : W / 8;   // column groups
    static constexpr int NITEM = 8 * CG;
    static_assert(NITEM <= 256, "one item per thread");
    const bf16_t *base;   // item's first load at step 0 (saved) or its column (row-major)
    int rp, cg;
    bool live;            // item index below NITEM
    __device__ WgOperand(const bf16_t *X, int c0, int ncol, int kbeg, int t)
    {
        live = t < NITEM;
        const int q = live ? t : 0;
        if (SAVED) {
            rp = q & 7;
            cg = q >> 3;
            // the step's 32 cells x W features are one run of the saved layout from
            // tm_idx(k, c0); item (rp, cg) is its 16-byte pieces 16 cg + 2 rp and + 1
            base = X + tm_idx(kbeg, c0) + 128 * cg + 16 * rp;
        } else {
            cg = q % CG;
            rp = q / CG;
            const int col = c0 + 8 * cg;
            base = X + (col < ncol ? col : 0);   // columns past the operand read its first ones
        }
    }
    // loads of step j (clamped to the last step je); rows past kend of a row-major operand
    // read row kend - 1
    __device__ __forceinline__ void load(int je, int kbeg, int kend, int ld, uint4 (&r)[4]) const
    {
        if (SAVED) {
            const bf16_t *p = base + (int64_t)je * 8192;   // 8192 elements per 32-cell group
            r[0] = *reinterpret_cast<const uint4 *>(p);
            r[1] = *reinterpret_cast<const uint4 *>(p + 8);
        } else {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int k = min(kbeg + 32 * je + 4 * rp + e, max(kend - 1, 0));
                r[e] = *reinterpret_cast<const uint4 *>(base + (int64_t)k * ld);
            }
        }
    }
    // clear rows at or past nvalid (relative to the step), then write the item's pair-dwords to
    // S[kp / 4][column][kp % 4] (STRIDE dwords per row)
    template <int STRIDE>
    __device__ __forceinline__ void store(unsigned *S, int nvalid, uint4 (&r)[4]) const
    {
        if (!live) return;
        if (nvalid < 32) {
            const int k0 = 4 * rp;
            if (SAVED) {
                if (k0 >= nvalid) r[0].x = r[0].y = 0u;
                if (k0 + 1 >= nvalid) r[0].z = r[0].w = 0u;
                if (k0 + 2 >= nvalid) r[1].x = r[1].y = 0u;
                if (k0 + 3 >= nvalid) r[1].z = r[1].w = 0u;
            } else {
#pragma unroll
                for (int e = 0; e < 4; e++)
                    if (k0 + e >= nvalid) r[e] = make_uint4(0, 0, 0, 0);
            }
        }
        unsigned *row = S + (rp >> 1) * STRIDE + 2 * (rp & 1);   // k pairs 2 rp, 2 rp + 1
        if (SAVED) {
            const uint4 a = kw_interleave4(r[0]), b = kw_interleave4(r[1]);
            uint2 *d = reinterpret_cast<uint2 *>(row + 4 * (4 * cg));
            d[0] = make_uint2(a.x, b.x);
            d[2] = make_uint2(a.y, b.y);
            d[4] = make_uint2(a.z, b.z);
            d[6] = make_uint2(a.w, b.w);
        } else {
            uint4 e0, e1, o0, o1;
            kw_interleave(r[0], r[1], e0, e1);   // k pair 2 rp, columns 0..3 and 4..7
            kw_interleave(r[2], r[3], o0, o1);   // k pair 2 rp + 1
            uint2 *d = reinterpret_cast<uint2 *>(row + 4 * (8 * cg));
            d[0] = make_uint2(e0.x, o0.x);
            d[2] = make_uint2(e0.y, o0.y);
            d[4] = make_uint2(e0.z, o0.z);
            d[6] = make_uint2(e0.w, o0.w);
            d[8] = make_uint2(e1.x, o1.x);
            d[10] = make_uint2(e1.y, o1.y);
            d[12] = make_uint2(e1.z, o1.z);
            d[14] = make_uint2(e1.w, o1.w);
        }
    }
};

// AT / BT: the operand is in the saved-array layout (tm_idx, width 256) rather than
// row-major [K][ld].
//
// One-dimensional grid of tiles_x * tiles_y * splits workgroups (splits a multiple of 8).
// Consecutive workgroups are dealt to the eight XCDs in turn, so workgroup b runs on XCD
// b % 8; the mapping gives every XCD whole batch splits (all tiles of split z on XCD z % 8),
// so the tiles that share an operand run side by side and read it through one L2.
//
// One launch covers every layer: the hidden layers (one shape), then the input and the output
// layer.  Within a shape group, workgroup b works on layer b / per_layer (per_layer a
// multiple of 8, so the XCD mapping within each layer is unchanged); the groups' block ranges
// follow each other, the long hidden-layer workgroups first, so the layers fill the machine
// together instead of each launch ending on its own tail.
struct WgGroup {
    const bf16_t *A[MAX_HIDDEN];
    const bf16_t *B[MAX_HIDDEN];
    float *C[MAX_HIDDEN];   // partials of split z at C + z strideC, the bias row right after
    int per_layer, end;     // workgroups per layer; the group's block range ends at `end`
    int lda, M, ldb, N, K, kchunk, tiles_x, tiles_y, ldc;
    int64_t strideC;
};
struct WgLaunch {
    WgGroup g[3];           // hidden layers, input layer, output layer
};

template <int TM, int TN, int WAVES_M, bool AT, bool BT, int DEPTH>
__device__ __forceinline__ void wgrad_tile(const WgGroup &G, int b, unsigned *lds)
{
    const int per_layer = G.per_layer, lda = G.lda, M = G.M, ldb = G.ldb, N = G.N, K = G.K;
    const int kchunk = G.kchunk, tiles_x = G.tiles_x, tiles_y = G.tiles_y, ldc = G.ldc;
    const int64_t strideC = G.strideC;
    const int layer = b / per_layer;
    const bf16_t *A = G.A[layer], *B = G.B[layer];
    float *C = G.C[layer], *Cb = C + (int64_t)M * ldc;
    constexpr int WAVES_N = 4 / WAVES_M;
    constexpr int BM = TM / WAVES_M / 32, BN = TN / WAVES_N / 32;
    static_assert(BM >= 1 && BN >= 1, "each wave holds at least one 32 x 32 block");
    constexpr int SA = 4 * (TM + KW_PAD), SB = 4 * (TN + KW_PAD);   // dwords per LDS row (8 k)
    unsigned(*As)[4 * SA] = reinterpret_cast<unsigned(*)[4 * SA]>(lds);
    unsigned(*Bs)[4 * SB] = reinterpret_cast<unsigned(*)[4 * SB]>(lds + 2 * 4 * SA);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w / WAVES_N, wn = w % WAVES_N;
    const int h = lane >> 5, r = lane & 31;
    const int ntile = tiles_x * tiles_y;
    const int bid = b - layer * per_layer, slot = bid >> 3;
    const int tile = slot % ntile, split = (slot / ntile) * 8 + (bid & 7);
    const int bx = tile % tiles_x, by = tile / tiles_x;
    const int m0 = by * TM, n0 = bx * TN;
    const int kbeg = split * kchunk;
    if (split > 0 && kbeg >= K) return;   // grid rounded up to whole splits per XCD
    const int kend = min(K, kbeg + kchunk);
    const int nsteps = kend > kbeg ? (kend - kbeg + 31) / 32 : 0;
    const int jlast = max(nsteps - 1, 0);
    const WgOperand<TM, AT> opA(A, m0, M, kbeg, t);
    const WgOperand<TN, BT> opB(B, n0, N, kbeg, t);

    f32x16 acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; i++)
#pragma unroll
        for (int j = 0; j < BN; j++) acc[i][j] = f32x16{};
    // bias gradient: the waves of the first column of the first column tile multiply their A
    // fragments by ones
    const bool colsum = Cb && bx == 0 && wn == 0;
    f32x16 accb[BM];
#pragma unroll
    for (int i = 0; i < BM; i++) accb[i] = f32x16{};
    const bf16x8 ones = __builtin_bit_cast(bf16x8, make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u));
    auto compute = [&](int buf) {
#pragma unroll
        for (int kb = 0; kb < 2; kb++) {
            const int kq = 2 * kb + h;   // this lane's k = 16 kb + 8 h .. + 7: LDS row kq
            bf16x8 af[BM], bfr[BN];
#pragma unroll
            for (int i = 0; i < BM; i++)
                af[i] = *reinterpret_cast<const bf16x8 *>(&As[buf][kq * SA + 4 * ((wm * BM + i) * 32 + r)]);
#pragma unroll
            for (int i = 0; i < BN; i++)
                bfr[i] = *reinterpret_cast<const bf16x8 *>(&Bs[buf][kq * SB + 4 * ((wn * BN + i) * 32 + r)]);
#pragma unroll
            for (int i = 0; i < BM; i++)
#pragma unroll
                for (int j = 0; j < BN; j++) acc[i][j] = mfma32(af[i], bfr[j], acc[i][j]);
            if (colsum) {
#pragma unroll
                for (int i = 0; i < BM; i++) accb[i] = mfma32(af[i], ones, accb[i]);
            }
        }
    };
    // Step j sits in LDS buffer j % 2 and, before that, in register set j % DEPTH: while step
    // j's MFMAs run, the loads of steps j + 1 .. j + DEPTH are in flight (each step waits for
    // its own loads only, which the in-order vmcnt allows), since one step's work is far
    // shorter than a load's latency.  Steps past the range load the last step again and clear
    // it at the store, so that no load sits in a branch.  The barrier waits for this wave's LDS
    // accesses only; a fenced __syncthreads would also drain the loads in flight.
    auto lds_barrier = [] {
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0); vmcnt and expcnt left alone
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    auto load = [&](int j, uint4 (&ra)[4], uint4 (&rb)[4]) {
        const int je = min(j, jlast);
        opA.load(je, kbeg, kend, lda, ra);
        opB.load(je, kbeg, kend, ldb, rb);
    };
    auto store = [&](int buf, int j, uint4 (&ra)[4], uint4 (&rb)[4]) {
        const int nvalid = kend - (kbeg + 32 * j);
        opA.template store<SA>(As[buf], nvalid, ra);
        opB.template store<SB>(Bs[buf], nvalid, rb);
    };
    // The loop is unrolled DEPTH times, so that the register set (j % DEPTH) and the LDS buffer
    // (j % 2) are constants, and runs whole rounds: the steps added at the end are cleared
    // (both operands zero) and add exact zeros.  A branch inside the round would make the
    // compiler move the accumulators at every iteration and drain the loads.
    static_assert(DEPTH % 2 == 0, "an even prefetch depth keeps the LDS buffer of a step constant");
    uint4 ra[DEPTH][4], rb[DEPTH][4];
#pragma unroll
    for (int d = 0; d < DEPTH; d++) load(d, ra[d], rb[d]);
    store(0, 0, ra[0], rb[0]);
    lds_barrier();
    for (int j0 = 0; j0 < nsteps; j0 += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; d++) {
            const int j = j0 + d;
            load(j + DEPTH, ra[d], rb[d]);
            compute(d & 1);
            store((d + 1) & 1, j + 1, ra[(d + 1) % DEPTH], rb[(d + 1) % DEPTH]);
            lds_barrier();
        }
    }
    // C layout of the 32 x 32 blocks: column = lane % 32 (n), rows 8q + 4h + (0..3) (m); every
    // column of a ones product holds the same sums
    if (colsum && r == 0) {
#pragma unroll
        for (int i = 0; i < BM; i++)
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int m = m0 + (wm * BM + i) * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
                if (m < M) Cb[split * strideC + m] = accb[i][v];
            }
    }
    float *Cz = C + split * strideC;
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

// the three tile shapes: hidden layers 128 x 128 (2 x 2 waves), input layer 128 x 32 (4 x 1),
// output layer 32 x 128 (1 x 4); LDS for the largest (two buffers of A and B rows)
constexpr int WG_LDS_DWORDS = 2 * 4 * 4 * (128 + KW_PAD) * 2;
__global__ __launch_bounds__(256) void gemm_wgrad_kernel(WgLaunch P)
{
    __shared__ __attribute__((aligned(16))) unsigned lds[WG_LDS_DWORDS];
    const int b = blockIdx.x;
    if (b < P.g[0].end) wgrad_tile<128, 128, 2, true, true, WG_DEPTH>(P.g[0], b, lds);
    else if (b < P.g[1].end) wgrad_tile<128, 32, 4, true, false, WG_DEPTH>(P.g[1], b - P.g[0].end, lds);
    else wgrad_tile<32, 128, 1, false, true, WG_DEPTH>(P.g[2], b - P.g[1].end, lds);
}

}  // namespace props

using namespace props;

// ------------------------------------------------------------------ the handle
struct props_dnn_s {
    int device = 0;
    int nhid = 4, nout = NOUT;
    float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;   // device FP32
    bf16_t *fused = nullptr, *bwd = nullptr;
    double *scal = nullptr;        // device: in_lo[10], in_inv[10], out_lo[6], out_rng[6], out_inv[6]
    double in_lo[NIN], in_hi[NIN], out_lo[NOUT], out_hi[NOUT];
    unsigned logmask = kPTYLogMask;   // outputs trained on their logarithm
    int64_t step = 0;
    int epoch = 0;
    // forward/backward scratch for one batch
    bf16_t *h0 = nullptr, *zs[MAX_HIDDEN] = {}, *hs[MAX_HIDDEN] = {}, *dzo = nullptr;
    float *part = nullptr, *lpart = nullptr;
    GradParts gp{};   // where the last fwd_bwd left each layer's partials
    int *fb_idx = nullptr, *fb_count = nullptr;
    int64_t fb_cap = 0;
    size_t params() const { return total_params(nhid); }
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
    hipLaunchKernelGGL(convert_weights_kernel, dim3(64, d->nhid + 1), dim3(256), 0, s, d->master, d->fused,
                       d->bwd, d->nhid);
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
    void *ps[] = {d->master, d->grad, d->m, d->v, d->fused, d->bwd, d->scal, d->h0, d->dzo,
                  d->part, d->lpart, d->fb_idx, d->fb_count};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    if (d->zs[0]) (void)hipFree(d->zs[0]);
    if (d->hs[0]) (void)hipFree(d->hs[0]);
    delete d;
}

static int alloc_dnn(props_dnn_s *d)
{
    int rc;
    const size_t P = d->params();
    if ((rc = dalloc(&d->master, P)) || (rc = dalloc(&d->grad, P)) || (rc = dalloc(&d->m, P)) ||
        (rc = dalloc(&d->v, P)) ||
        (rc = dalloc(&d->fused, f_total(d->nhid))) || (rc = dalloc(&d->bwd, bf_total(d->nhid))) ||
        (rc = dalloc(&d->scal, (size_t)NIN * 2 + NOUT * 3)) ||
        (rc = dalloc(&d->fb_count, 1)))
        return rc;
    PROPS_HIP_TRY(hipMemset(d->grad, 0, P * sizeof(float)));
    PROPS_HIP_TRY(hipMemset(d->m, 0, P * sizeof(float)));
    PROPS_HIP_TRY(hipMemset(d->v, 0, P * sizeof(float)));
    PROPS_HIP_TRY(hipMemset(d->fused, 0, f_total(d->nhid) * sizeof(bf16_t)));
    PROPS_HIP_TRY(hipMemset(d->bwd, 0, bf_total(d->nhid) * sizeof(bf16_t)));
    return PROPS_OK;
}

static int ensure_train_scratch(props_dnn_s *d)
{
    if (d->h0) return PROPS_OK;
    int rc;
    const size_t B = MAX_BATCH;
    if ((rc = dalloc(&d->h0, B * IN_PAD)) ||
        (rc = dalloc(&d->dzo, B * OUT_PAD)) ||
        (rc = dalloc(&d->part, part_floats(d->nhid))) ||
        (rc = dalloc(&d->lpart, (size_t)B / CELLS_PER_WAVE + 64)))
        return rc;
    // the forward writes input columns 0..15 of the saved inputs; 16..31 stay zero
    PROPS_HIP_TRY(hipMemset(d->h0, 0, sizeof(bf16_t) * B * IN_PAD));
    // the hidden layers' saves, one block each, layer l at offset l B 256
    if ((rc = dalloc(&d->hs[0], B * HID * d->nhid)) || (rc = dalloc(&d->zs[0], B * HID * d->nhid))) return rc;
    for (int l = 1; l < d->nhid; l++) d->hs[l] = d->hs[0] + l * B * HID, d->zs[l] = d->zs[0] + l * B * HID;
    return PROPS_OK;
}

// One workgroup per CU, capped by the tile count.
static int fwd_grid(int64_t n)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    const int64_t tiles = (n + TILE_CELLS - 1) / TILE_CELLS;
    return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)cus));
}

static std::once_flag g_bwd_lds_once;
static hipError_t g_bwd_lds_err = hipSuccess;
static int launch_bwd(const BwdArgs &b, hipStream_t s)
{
    std::call_once(g_bwd_lds_once, [] {
        g_bwd_lds_err = hipFuncSetAttribute((const void *)mlp_bwd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            BWD_LDS_BYTES);
    });
    if (g_bwd_lds_err != hipSuccess)
        return fail(PROPS_EHIP, "hipFuncSetAttribute(LDS %d B): %s", BWD_LDS_BYTES, hipGetErrorString(g_bwd_lds_err));
    hipLaunchKernelGGL(mlp_bwd_kernel, dim3(fwd_grid(b.n)), dim3(FWD_THREADS), BWD_LDS_BYTES, s, b);
    PROPS_HIP_TRY(hipGetLastError());
    return PROPS_OK;
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

// dW = dz^T h (and db = column sums of dz) for the layer shapes of the network: (256, 256) on
// 128 x 128 tiles in SPLIT_HID batch splits, (256, 32) (input layer) on 128 x 32 tiles and
// (16, 256) (output layer) on 32 x 128 tiles in SPLIT_IO splits.  Split z writes its W
// partials at part + z (O I + O) and its bias partials right after them, so one ordered
// reduction gives W and b, which are adjacent in the master.
static int wgrad_nsplit(int O, int I) { return (O % 128 == 0 && I % 128 == 0) ? SPLIT_HID : SPLIT_IO; }

// the number of batch splits of a layer of O x I on n rows
static int wgrad_splits(int O, int I, int n)
{
    const int nsplit = wgrad_nsplit(O, I);
    const int kchunk = ((n + nsplit - 1) / nsplit + 31) / 32 * 32;
    return (n + kchunk - 1) / kchunk;
}

// the shape group of nl layers of O x I (tiles TM x TN) whose block range starts at `start`
static void wgrad_group(WgGroup &G, int nl, int O, int I, int TM, int TN, int n, int start)
{
    const int nsplit = wgrad_nsplit(O, I);
    G.kchunk = ((n + nsplit - 1) / nsplit + 31) / 32 * 32;
    const int splits = (n + G.kchunk - 1) / G.kchunk;
    G.tiles_x = (I + TN - 1) / TN;
    G.tiles_y = (O + TM - 1) / TM;
    G.per_layer = G.tiles_x * G.tiles_y * ((splits + 7) / 8 * 8);
    G.end = start + G.per_layer * nl;
    G.lda = O, G.M = O, G.ldb = I, G.N = I, G.K = n, G.ldc = I;
    G.strideC = (int64_t)O * I + O;
}

// The training set as rows of SAMPLE_FLOATS floats (inputs, targets, zeros): the epoch
// permutation then reads one 64-byte row per sample instead of a 4-byte value from each of the
// sixteen feature-major rows (sixteen cache lines).
__global__ void pack_samples_kernel(const float *X, const float *Y, int64_t n, int nout, float *XY)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v[SAMPLE_FLOATS];
#pragma unroll
    for (int f = 0; f < SAMPLE_FLOATS; f++) {
        const int j = f - NIN;
        v[f] = f < NIN ? X[(int64_t)f * n + i] : j < nout ? Y[(int64_t)j * n + i] : 0.0f;
    }
    float4 *dst = reinterpret_cast<float4 *>(XY + SAMPLE_FLOATS * i);
#pragma unroll
    for (int q = 0; q < SAMPLE_FLOATS / 4; q++) dst[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}

// frees a device allocation when the entry point returns (hipFree waits for the device)
struct DevFree {
    void *p;
    ~DevFree()
    {
        if (p) (void)hipFree(p);
    }
};

static int pack_samples(const float *X, const float *Y, int64_t n, int nout, float **xy, hipStream_t s)
{
    int rc;
    if ((rc = dalloc(xy, (size_t)n * SAMPLE_FLOATS))) return rc;
    hipLaunchKernelGGL(pack_samples_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, Y, n, nout, *xy);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        (void)hipFree(*xy);
        *xy = nullptr;
        return fail(PROPS_EHIP, "pack_samples: %s", hipGetErrorString(e));
    }
    return PROPS_OK;
}

// One forward + backward pass over rows [row0, row0 + n) of the permuted data; leaves each
// layer's split-K gradient partials (d->gp, reduced by grad_step) and the loss partials (one
// per wave of 32 rows) in lpart.
static int fwd_bwd(props_dnn_s *d, const float *XY, int64_t nx, uint64_t pa, uint64_t pc, int64_t row0, int n,
                   float *lpart, hipStream_t s)
{
    int rc;
    const int nh = d->nhid;
    FwdArgs a{};
    a.XY = XY;
    a.nx = nx;
    a.pa = pa;
    a.pc = pc;
    a.row0 = row0;
    a.n = n;
    a.nhid = nh;
    a.nout = d->nout;
    a.Wf = d->fused;
    a.in_lo = d->scal;
    a.in_inv = d->scal + NIN;
    a.out_lo = d->scal + 2 * NIN;
    a.out_inv = d->scal + 2 * NIN + 2 * NOUT;
    a.logmask = d->logmask;
    a.h0 = d->h0;
    a.zs = d->zs[0];
    a.hs = d->hs[0];
    a.lstride = (int64_t)MAX_BATCH * HID;
    a.dzo = d->dzo;
    a.lpart = lpart;
    if ((rc = launch_fwd(true, a, s))) return rc;
    // dz of every hidden layer in one fused pass, written over the saved z
    BwdArgs bw{};
    bw.Wb = d->bwd;
    bw.dzo = d->dzo;
    bw.zs = d->zs[0];
    bw.lstride = (int64_t)MAX_BATCH * HID;
    bw.n = n;
    bw.nhid = nh;
    if ((rc = launch_bwd(bw, s))) return rc;
    // weight and bias gradients, output layer to input: dW_l = dz_l^T h_{l-1}, db_l = sum dz_l
    // (M = O, N = I, K = n), split over the batch; the partials stay for grad_step, laid out
    // output layer first
    float *pl = d->part, *lpart_of[MAX_HIDDEN + 1];
    d->gp.nl = nh + 1;
    for (int l = 0; l <= nh; l++) d->gp.off[l] = (int64_t)w_off(l);
    d->gp.off[nh + 1] = (int64_t)total_params(nh);
    for (int l = nh; l >= 0; l--) {
        const int O = lout(l, nh), I = lin(l);
        d->gp.part[l] = lpart_of[l] = pl;
        d->gp.splits[l] = wgrad_splits(O, I, n);
        pl += (size_t)d->gp.splits[l] * ((size_t)O * I + O);
    }
    // one launch: the hidden layers (both operands in the saved-array layout), the input layer
    // (dz saved, the inputs row-major [n][32]), the output layer (dz row-major [n][16], h saved)
    WgLaunch P{};
    for (int l = nh - 1, j = 0; l >= 1; l--, j++) {
        P.g[0].A[j] = d->zs[l];
        P.g[0].B[j] = d->hs[l - 1];
        P.g[0].C[j] = lpart_of[l];
    }
    wgrad_group(P.g[0], nh - 1, HID, HID, 128, 128, n, 0);
    P.g[1].A[0] = d->zs[0];
    P.g[1].B[0] = d->h0;
    P.g[1].C[0] = lpart_of[0];
    wgrad_group(P.g[1], 1, HID, IN_PAD, 128, 32, n, P.g[0].end);
    P.g[2].A[0] = d->dzo;
    P.g[2].B[0] = d->hs[nh - 1];
    P.g[2].C[0] = lpart_of[nh];
    wgrad_group(P.g[2], 1, OUT_PAD, HID, 32, 128, n, P.g[1].end);
    static_assert(IN_PAD == 32 && OUT_PAD <= 32 && OUT_PAD % 8 == 0 && HID % 128 == 0,
                  "the three tile shapes of gemm_wgrad_kernel");
    hipLaunchKernelGGL(gemm_wgrad_kernel, dim3(P.g[2].end), dim3(256), 0, s, P);
    PROPS_HIP_TRY(hipGetLastError());
    return PROPS_OK;
}

// The reduction of the last fwd_bwd's partials: into d->grad (adam = false), or straight
// into an Adam step of the master and its bf16 copies.
static int grad_step(props_dnn_s *d, bool adam, float lr, float b1, float b2, float eps, float bc1, float bc2,
                     hipStream_t s)
{
    const int64_t P = d->gp.off[d->gp.nl];
    const int64_t threads = P / GS_VEC * GS_LANES;
    hipLaunchKernelGGL(grad_step_kernel, dim3((unsigned)((threads + GS_THREADS - 1) / GS_THREADS)), dim3(GS_THREADS), 0, s, d->gp, d->nhid, d->grad,
                       d->master, d->m, d->v, d->fused, d->bwd, (int)adam, lr, b1, b2, eps, bc1, bc2);
    PROPS_HIP_TRY(hipGetLastError());
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
    if (d->logmask != kPTYLogMask || d->nout != NOUT)
        return fail(PROPS_EINVAL, "props_dnn: the network (%d outputs, log mask 0x%x) is not one of (rho, h, cp, "
                    "c, mu, lambda); evaluate it with props_dnn_features", d->nout, d->logmask);
    if (fb && fb->ns != NIN - 2)
        return fail(PROPS_EINVAL, "props_dnn: fallback mechanism has %d species, the network %d", fb->ns, NIN - 2);
    if (fb && (!fb_idx || !fb_count)) return fail(PROPS_EINVAL, "props_dnn: fallback needs index scratch");
    int rc;
    FwdArgs a{};
    a.P = in->P, a.T = in->T, a.Y = in->Y, a.n = n, a.ldy = ldy;
    a.nhid = d->nhid, a.nout = d->nout;
    a.Wf = d->fused;
    a.in_lo = d->scal, a.in_inv = d->scal + NIN;
    a.out_lo = d->scal + 2 * NIN, a.out_rng = d->scal + 2 * NIN + NOUT;
    a.logmask = d->logmask;
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

static int fit_scalers_dev(props_dnn_s *d, const float *X, const float *Y, int64_t n, hipStream_t s)
{
    const int B = 256;
    const int64_t per = (n + B - 1) / B;
    double *part = nullptr;
    int rc;
    const int no = d->nout;
    if ((rc = dalloc(&part, (size_t)B * 2 * (NIN + no)))) return rc;
    hipLaunchKernelGGL(minmax_partial_kernel, dim3(B, NIN), dim3(256), 0, s, X, n, NIN, 0u, per, part);
    hipLaunchKernelGGL(minmax_partial_kernel, dim3(B, no), dim3(256), 0, s, Y, n, no, d->logmask, per,
                       part + (size_t)B * 2 * NIN);
    std::vector<double> h((size_t)B * 2 * (NIN + no));
    hipError_t e = hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(part);
    if (e != hipSuccess) return fail(PROPS_EHIP, "fit scalers: %s", hipGetErrorString(e));
    for (int f = 0; f < NIN + no; f++) {
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

static double loss_of(const std::vector<float> &lp, int64_t rows, int nout)
{
    double sl = 0;
    for (float v : lp) sl += v;
    return sl / ((double)rows * nout);
}

}  // namespace props

extern "C" {

int props_dnn_create_ex(uint64_t seed, int hidden_layers, int outputs, props_dnn_t *out)
{
    if (!out) return fail(PROPS_EINVAL, "props_dnn_create: out is NULL");
    *out = nullptr;
    if (hidden_layers < MIN_HIDDEN || hidden_layers > MAX_HIDDEN)
        return fail(PROPS_EINVAL, "props_dnn_create: %d hidden layers (%d or %d supported)", hidden_layers, MIN_HIDDEN,
                    MAX_HIDDEN);
    if (outputs < 1 || outputs > NOUT) return fail(PROPS_EINVAL, "props_dnn_create: %d outputs (1..%d)", outputs, NOUT);
    props_dnn_s *d = new (std::nothrow) props_dnn_s();
    if (!d) return fail(PROPS_ENOMEM, "props_dnn_create: out of host memory");
    d->nhid = hidden_layers;
    d->nout = outputs;
    if (hipGetDevice(&d->device) != hipSuccess) {
        delete d;
        return fail(PROPS_EHIP, "props_dnn_create: hipGetDevice failed");
    }
    int rc = alloc_dnn(d);
    if (rc) {
        free_dnn(d);
        return rc;
    }
    const int nh = d->nhid;
    std::vector<float> h(d->params(), 0.0f);
    uint64_t st = seed;
    for (int l = 0; l <= nh; l++) {
        const double k = 1.0 / std::sqrt((double)tin(l));
        const int to = tout(l, nh, d->nout);
        for (int o = 0; o < to; o++)
            for (int i = 0; i < tin(l); i++) h[w_off(l) + (size_t)o * lin(l) + i] = (float)((2.0 * u01(st) - 1.0) * k);
        for (int o = 0; o < to; o++) h[b_off(l, nh) + o] = (float)((2.0 * u01(st) - 1.0) * k);
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

int props_dnn_create(uint64_t seed, props_dnn_t *out) { return props_dnn_create_ex(seed, 4, NOUT, out); }

void props_dnn_destroy(props_dnn_t net)
{
    if (net) free_dnn(net);
}

int props_dnn_get_shape(props_dnn_t d, int *hidden_layers, int *outputs)
{
    if (!d) return fail(PROPS_EINVAL, "props_dnn_get_shape: null network");
    if (hidden_layers) *hidden_layers = d->nhid;
    if (outputs) *outputs = d->nout;
    return PROPS_OK;
}

int props_dnn_get_layer(props_dnn_t d, int l, float *W, float *b)
{
    if (!d || l < 0 || l > d->nhid) return fail(PROPS_EINVAL, "props_dnn_get_layer: bad network or layer");
    const int nh = d->nhid, to = tout(l, nh, d->nout);
    std::vector<float> h((size_t)lout(l, nh) * lin(l) + lout(l, nh));
    PROPS_HIP_TRY(hipMemcpy(h.data(), d->master + w_off(l), h.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (int o = 0; o < to; o++) {
        if (W)
            for (int i = 0; i < tin(l); i++) W[(size_t)o * tin(l) + i] = h[(size_t)o * lin(l) + i];
        if (b) b[o] = h[(size_t)lout(l, nh) * lin(l) + o];
    }
    return PROPS_OK;
}

int props_dnn_set_layer(props_dnn_t d, int l, const float *W, const float *b)
{
    if (!d || l < 0 || l > d->nhid || !W || !b) return fail(PROPS_EINVAL, "props_dnn_set_layer: bad arguments");
    const int nh = d->nhid, to = tout(l, nh, d->nout);
    std::vector<float> h((size_t)lout(l, nh) * lin(l) + lout(l, nh), 0.0f);
    for (int o = 0; o < to; o++) {
        for (int i = 0; i < tin(l); i++) h[(size_t)o * lin(l) + i] = W[(size_t)o * tin(l) + i];
        h[(size_t)lout(l, nh) * lin(l) + o] = b[o];
    }
    PROPS_HIP_TRY(hipMemcpy(d->master + w_off(l), h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    PROPS_HIP_TRY(hipMemset(d->m + w_off(l), 0, h.size() * sizeof(float)));
    PROPS_HIP_TRY(hipMemset(d->v + w_off(l), 0, h.size() * sizeof(float)));
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
    a.nhid = d->nhid, a.nout = d->nout;
    a.Wf = d->fused;
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

int props_dnn_grad(props_dnn_t d, const float *X, const float *Y, int64_t n, float *grad, float *loss,
                   void *hip_stream)
{
    ApiRange range_("props_dnn_grad");
    if (!d || !X || !Y || !grad) return fail(PROPS_EINVAL, "props_dnn_grad: null argument");
    if (n < 1 || n > MAX_BATCH) return fail(PROPS_EINVAL, "props_dnn_grad: need 1 <= n <= %d", MAX_BATCH);
    hipStream_t s = (hipStream_t)hip_stream;
    int rc;
    if ((rc = ensure_train_scratch(d))) return rc;
    float *xy = nullptr;
    if ((rc = pack_samples(X, Y, n, d->nout, &xy, s))) return rc;
    const DevFree xy_free{xy};
    if ((rc = fwd_bwd(d, xy, n, 1, 0, 0, (int)n, d->lpart, s))) return rc;
    if ((rc = grad_step(d, false, 0.f, 0.f, 0.f, 0.f, 1.f, 1.f, s))) return rc;
    const int nh = d->nhid;
    const size_t nw = (size_t)((n + TILE_CELLS - 1) / TILE_CELLS) * FWD_WAVES;
    std::vector<float> g(d->params()), lp(nw);
    PROPS_HIP_TRY(hipMemcpyAsync(g.data(), d->grad, g.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    PROPS_HIP_TRY(hipMemcpyAsync(lp.data(), d->lpart, lp.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    PROPS_HIP_TRY(hipStreamSynchronize(s));
    size_t o = 0;
    for (int l = 0; l <= nh; l++) {
        const int to = tout(l, nh, d->nout);
        for (int r = 0; r < to; r++)
            for (int i = 0; i < tin(l); i++) grad[o++] = g[w_off(l) + (size_t)r * lin(l) + i];
        for (int r = 0; r < to; r++) grad[o++] = g[b_off(l, nh) + r];
    }
    if (loss) *loss = (float)loss_of(lp, n, d->nout);
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
    float *xy = nullptr;
    if ((rc = pack_samples(X, Y, n, d->nout, &xy, s))) return rc;
    const DevFree xy_free{xy};
    const int total = cfg->total_epochs > 0 ? cfg->total_epochs : std::max(1, d->epoch + cfg->epochs);
    const float b1 = cfg->beta1 > 0 ? cfg->beta1 : 0.9f, b2 = cfg->beta2 > 0 ? cfg->beta2 : 0.999f;
    const float eps = cfg->eps > 0 ? cfg->eps : 1e-8f;
    const int64_t steps_per_epoch = (n + batch - 1) / batch;
    std::vector<float> lp;
    int64_t steps = 0;
    float *lsum = nullptr;   // per-step loss partials of one epoch (one per wave of 32 rows)
    const int lslots = batch / CELLS_PER_WAVE;
    if ((rc = dalloc(&lsum, (size_t)steps_per_epoch * lslots))) return rc;
    for (int e = 0; e < cfg->epochs; e++) {
        uint64_t pa, pc;
        epoch_perm(cfg->seed, d->epoch, n, pa, pc);
        const double prog = std::min(1.0, (double)d->epoch / total);
        hipLaunchKernelGGL(fill_float_kernel, dim3((unsigned)((steps_per_epoch * lslots + 255) / 256)), dim3(256), 0, s,
                           lsum, steps_per_epoch * lslots, 0.0f);
        const float lr = (float)(cfg->lr_min + 0.5 * (cfg->lr - cfg->lr_min) * (1.0 + std::cos(M_PI * prog)));
        for (int64_t st = 0; st < steps_per_epoch; st++) {
            const int64_t row0 = st * batch;
            const int m = (int)std::min<int64_t>(batch, n - row0);
            // the loss partials go straight to this step's slots of the epoch's array
            if ((rc = fwd_bwd(d, xy, n, pa, pc, row0, m, lsum + st * lslots, s))) {
                (void)hipFree(lsum);
                return rc;
            }
            d->step++;
            const float bc1 = 1.0f - std::pow(b1, (float)d->step), bc2 = 1.0f - std::pow(b2, (float)d->step);
            if ((rc = grad_step(d, true, lr, b1, b2, eps, bc1, bc2, s))) {
                (void)hipFree(lsum);
                return rc;
            }
            steps++;
        }
        lp.resize((size_t)steps_per_epoch * lslots);
        hipError_t err = hipMemcpyAsync(lp.data(), lsum, lp.size() * sizeof(float), hipMemcpyDeviceToHost, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        if (err != hipSuccess) {
            (void)hipFree(lsum);
            return fail(PROPS_EHIP, "train_dnn: %s", hipGetErrorString(err));
        }
        if (rep && rep->loss) rep->loss[e] = (float)loss_of(lp, n, d->nout);
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

// ---- checkpoint: "PROPSDNN" v3 | params | step | epoch | log-output mask | hidden layers |
// outputs | scalers | master | m | v  (v1, v2: the 4-layer, 6-output network; v1 without the
// mask loads with the (P, T, Y) surrogate's mask)
int props_dnn_save(props_dnn_t d, const char *path)
{
    ApiRange range_("props_dnn_save");
    if (!d || !path) return fail(PROPS_EINVAL, "props_dnn_save: null argument");
    const size_t P = d->params();
    std::vector<float> buf(3 * P);
    PROPS_HIP_TRY(hipDeviceSynchronize());
    PROPS_HIP_TRY(hipMemcpy(buf.data(), d->master, P * 4, hipMemcpyDeviceToHost));
    PROPS_HIP_TRY(hipMemcpy(buf.data() + P, d->m, P * 4, hipMemcpyDeviceToHost));
    PROPS_HIP_TRY(hipMemcpy(buf.data() + 2 * P, d->v, P * 4, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(PROPS_EINVAL, "props_dnn_save: cannot open %s", path);
    const char magic[8] = {'P', 'R', 'O', 'P', 'S', 'D', 'N', 'N'};
    const uint32_t ver = 3;
    const uint64_t np = P;
    const uint32_t mask = d->logmask;
    const int32_t shape[2] = {d->nhid, d->nout};
    bool ok = std::fwrite(magic, 8, 1, f) == 1 && std::fwrite(&ver, 4, 1, f) == 1 && std::fwrite(&np, 8, 1, f) == 1 &&
              std::fwrite(&d->step, 8, 1, f) == 1 && std::fwrite(&d->epoch, 4, 1, f) == 1 &&
              std::fwrite(&mask, 4, 1, f) == 1 && std::fwrite(shape, 4, 2, f) == 2 &&
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
    int64_t step = 0;
    int32_t epoch = 0;
    uint32_t mask = kPTYLogMask;
    int32_t shape[2] = {4, NOUT};
    bool ok = std::fread(magic, 8, 1, f) == 1 && std::memcmp(magic, "PROPSDNN", 8) == 0 && std::fread(&ver, 4, 1, f) == 1 &&
              (ver >= 1 && ver <= 3) && std::fread(&np, 8, 1, f) == 1 && std::fread(&step, 8, 1, f) == 1 &&
              std::fread(&epoch, 4, 1, f) == 1 && (ver == 1 || std::fread(&mask, 4, 1, f) == 1) &&
              (ver < 3 || std::fread(shape, 4, 2, f) == 2) && (mask >> NOUT) == 0;
    props_dnn_t d = nullptr;
    int rc = PROPS_OK;
    if (ok) {
        rc = props_dnn_create_ex(0, shape[0], shape[1], &d);
        ok = rc == PROPS_OK && np == d->params();
    }
    std::vector<float> buf;
    if (ok) {
        buf.resize(3 * np);
        ok = std::fread(d->in_lo, sizeof(d->in_lo), 1, f) == 1 && std::fread(d->in_hi, sizeof(d->in_hi), 1, f) == 1 &&
             std::fread(d->out_lo, sizeof(d->out_lo), 1, f) == 1 && std::fread(d->out_hi, sizeof(d->out_hi), 1, f) == 1 &&
             std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    }
    std::fclose(f);
    if (!ok) {
        if (d) props_dnn_destroy(d);
        return fail(rc ? rc : PROPS_EINVAL, "props_dnn_load: %s is not a valid checkpoint", path);
    }
    d->step = step;
    d->epoch = epoch;
    d->logmask = mask;
    const size_t P = np;
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
