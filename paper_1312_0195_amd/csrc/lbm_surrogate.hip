// lbm_surrogate.hip -- learned K_eff surrogate: BF16 MFMA forward and
// training kernels for gfx950.
//
// The network (not part of the paper) maps a periodic 32 x 32 log-permeability
// patch to log K_eff (xx and yy), the quantity the local problems of Sec. 3
// compute with Eq. tensor-kappa:
//   m = mean(log K), x = log K - m                    (FP32)
//   a1 = relu(conv3x3(x))      1 -> 32 channels      (BF16 MFMA, the 9 taps and zeros as K = 16)
//   a2..a4 = relu(conv3x3(.))  32 -> 32 channels     (BF16 MFMA, FP32 accumulate)
//   p = mean over pixels of a4                       (FP32)
//   s = log series/parallel estimates of exp(x)      (FP32, 4 values:
//       mean over rows of the harmonic mean along each row; harmonic mean over
//       columns of the arithmetic mean along each column; and the same with
//       rows and columns exchanged)
//   z = [p, m, s], h = relu(M1 z + c1), y = M2 h + c2, prediction = y + m
// A symmetry of the square can be applied to a patch as it is read (sym =
// t + 2 fx + 4 fy: transpose, then mirror x, then mirror y); a transposition
// exchanges the kxx and kyy outputs. Training draws one per patch (given by
// the caller); inference can average the prediction over all eight.
// Convolutions wrap periodically (the local problems are periodic), so the
// network is invariant to circular shifts of a patch.
//
// Parameters are one FP32 vector (layout below). Each launch converts the
// conv2-4 weights to BF16 in the two layouts the MFMA operands need.
//
// Forward: one workgroup (8 waves) per patch at a time, persistent over the
// batch. Activations stay in LDS ([pixel][channel] BF16 with the channel
// chunks of each pixel permuted (act_off), 64 KB per layer plus halo rows,
// two buffers), and the BF16 weights of the 32 -> 32 layers pass through an
// 18 KB LDS buffer, one layer ahead, loaded from global memory straight into
// LDS while a layer runs (as is the next pass's input); a 16x16x32 MFMA takes
// 16 pixels x 32 input channels of one tap, so a 3x3 layer is 9 MFMAs per
// 16-pixel x 16-channel output tile, and each wave reads every input row of
// its eight output rows once. No global read is waited for in line with the
// layers. The last conv layer is pooled straight from the accumulators.
//
// Training: the forward also stores a1..a4 (BF16) and the pooled features;
// the head backward runs per patch in FP32; the conv backward walks layers
// 4 -> 1 per patch with two LDS buffers (layer input and gradient), computing
//   dW[tap][ci][co] += sum_p X[p + tap][ci] dZ[p][co]        (MFMA, K = pixels)
//   dX[p][ci] = sum_tap,co dZ[p - tap][co] W[tap][ci][co]   (MFMA, K = channels)
// Weight gradients accumulate in FP32 registers per workgroup over its
// patches and are summed over workgroups in a fixed order, so results do not
// depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "lbm_internal.h"

// Scratch of lbm_cnn_forward_noalloc: what the inference workspace holds
// (the BF16 conv weights in both operand layouts and the patch counter), one
// copy per device, kept until the process ends. Host code never uses this
// name as an address: it takes the device address once per device with
// hipGetSymbolAddress and passes that to the kernels.
constexpr size_t kNoAllocScratchBytes = 128 * 1024;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace lbm {
namespace {

constexpr int kSide = 32;
constexpr int kPix = kSide * kSide;  // 1024
constexpr int kC = 32;               // channels
constexpr int kH = 32;               // hidden units of the head
constexpr int kT = 512;              // threads per workgroup
constexpr int kWaves = kT / 64;

// parameter layout (FP32 offsets)
constexpr int oW1 = 0, oB1 = oW1 + 9 * kC;                  // W1[tap][co]
constexpr int oW2 = oB1 + kC, oB2 = oW2 + 9 * kC * kC;       // W[tap][ci][co]
constexpr int oW3 = oB2 + kC, oB3 = oW3 + 9 * kC * kC;
constexpr int oW4 = oB3 + kC, oB4 = oW4 + 9 * kC * kC;
constexpr int kZ = kC + 5;                                     // head input size
constexpr int oM1 = oB4 + kC, oC1 = oM1 + kH * kZ;            // M1[h][37]
constexpr int oM2 = oC1 + kH, oC2 = oM2 + 2 * kH;             // M2[2][h]
constexpr int kNParams = oC2 + 2;
constexpr int kNConv = oM1;               // parameters of the conv layers
constexpr int kNHead = kNParams - oM1;    // parameters of the head

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wrap32(int v) { return v & (kSide - 1); }

// Element offset of the 8-channel chunk c (0..3) of pixel p in an activation
// buffer of the forward pass in LDS. The four 16-byte chunks of a pixel are
// permuted by (p >> 1) & 3: the layers read one chunk of 16 consecutive
// pixels per MFMA operand (one 16-byte read per lane), and without the
// permutation those reads, 64 bytes apart, fall on the same few banks. With
// it, any 8 consecutive pixels (also across the periodic wrap of a row) hit
// 8 different 16-byte bank groups. Global copies of the activations keep the
// plain [pixel][channel] order.
__device__ __forceinline__ int act_off(int p, int c) { return p * kC + ((c ^ ((p >> 1) & 3)) << 3); }

// The forward pass keeps one periodic halo row above and below each plane in
// LDS (row -1 = row 31, row 32 = row 0): an activation buffer is 34 rows of
// kSide * kC elements whose row 0 starts kSide * kC elements in (kActRow),
// and the centred input plane has kSide floats before and after it. With
// the halo a 3x3 stencil never wraps in y, so every operand read of a tile
// is a per-lane base plus a compile-time offset.
constexpr int kActRow = kSide * kC;               // elements per activation row
constexpr int kActElems = (kSide + 2) * kActRow;  // one buffer with its halo rows
__device__ __forceinline__ int tap_dy(int t) { return t / 3 - 1; }
__device__ __forceinline__ int tap_dx(int t) { return t % 3 - 1; }

// Input pixel read for output pixel p under symmetry sym.
__device__ __forceinline__ int sym_src(int p, int sym)
{
    int u = p & 31, v = p >> 5;
    if (sym & 1) {
        const int t = u;
        u = v;
        v = t;
    }
    if (sym & 2) u = 31 - u;
    if (sym & 4) v = 31 - v;
    return v * kSide + u;
}

// Sums over 8- and 16-lane groups with DPP lane moves (no LDS permutes):
// within a quad the moves pair lanes i and i ^ 1, then i ^ 2; the mirrors
// then pair each lane with one of the other half of its 8- or 16-lane group,
// which holds the same value as lane i ^ 4 (i ^ 8) once the halves are
// reduced, so the sums are bit for bit those of a xor butterfly over 1, 2,
// 4 (and 8).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float group_sum8(float v)
{
    v += dpp_mov<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    return v;
}
__device__ __forceinline__ float group_sum16(float v)
{
    v = group_sum8(v);
    v += dpp_mov<0x140>(v);  // row_mirror
    return v;
}
// A xor butterfly over the wave in the order 32, 16, 8, 4, 2, 1, bit for bit:
// the two steps across 16-lane rows as lane permutes, then a rotation of
// each row by 8 (lane i gets lane i ^ 8), by 4 (the row now repeats every 8
// lanes, so i + 4 has the value of i ^ 4), and the quad moves.
__device__ __forceinline__ float wave_sum_desc(float v)
{
    v += __shfl_xor(v, 32, 64);
    v += __shfl_xor(v, 16, 64);
    v += dpp_mov<0x128>(v);  // row_ror:8
    v += dpp_mov<0x124>(v);  // row_ror:4
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0xB1>(v);
    return v;
}
// Lane 0's value of a xor butterfly over 16 and 32 when every 16-lane row
// is uniform (or only the first lane of each row counts): (row 0 + row 1) +
// (row 2 + row 3), read from lanes 0, 16, 32, 48.
__device__ __forceinline__ float rows_sum_lane0(float v)
{
    const int b = __builtin_bit_cast(int, v);
    const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 16));
    const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 32));
    const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 48));
    return (v + r1) + (r2 + r3);
}

// The four series/parallel features of k = exp(x) from the centred patch in
// LDS, on all 512 threads: 8 threads per line (lines 0..31 rows, 32..63
// columns) each sum 1/k and k over 4 pixels; fixed-order butterflies give
// the line sums, then the sums over the 8 lines of each wave, then thread 0
// adds the waves (rows: waves 0..3, columns: 4..7). lane_tmp: 16 floats.
__device__ __forceinline__ void series_parallel(const float *xs, float *lane_tmp, float *feat)
{
    const int tid = threadIdx.x;
    const int line = tid >> 3, part = tid & 7, r = line & 31;
    float hs = 0.0f, as = 0.0f;  // sums of 1/k and k along the line
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = part * 4 + i;
        const float x = line < 32 ? xs[r * kSide + j] : xs[j * kSide + r];
        hs += __expf(-x);
        as += __expf(x);
    }
    hs = group_sum8(hs);
    as = group_sum8(as);
    float h = kSide / hs;   // harmonic mean of the line
    float ia = kSide / as;  // 1 / arithmetic mean of the line
    h += dpp_mov<0x140>(h);  // the 8-lane groups are uniform: the mirror pairs as i ^ 8 does
    ia += dpp_mov<0x140>(ia);
    h = rows_sum_lane0(h);  // lane 0 writes the wave's value below
    ia = rows_sum_lane0(ia);
    const int wave = tid >> 6;
    if ((tid & 63) == 0) {
        lane_tmp[wave] = h;
        lane_tmp[8 + wave] = ia;
    }
    __syncthreads();
    if (tid == 0) {
        const float rh = (lane_tmp[0] + lane_tmp[1]) + (lane_tmp[2] + lane_tmp[3]);    // rows: harmonic along x
        const float ch = (lane_tmp[4] + lane_tmp[5]) + (lane_tmp[6] + lane_tmp[7]);    // columns: harmonic along y
        const float ria = (lane_tmp[8] + lane_tmp[9]) + (lane_tmp[10] + lane_tmp[11]);  // rows: 1/arithmetic
        const float cia = (lane_tmp[12] + lane_tmp[13]) + (lane_tmp[14] + lane_tmp[15]);  // columns
        feat[0] = logf(rh / 32.0f);
        feat[1] = -logf(cia / 32.0f);
        feat[2] = logf(ch / 32.0f);
        feat[3] = -logf(ria / 32.0f);
    }
    __syncthreads();
}

__device__ __forceinline__ float block_sum_fixed(float v, float *red)
{
    // fixed-order sum over the workgroup: wave butterflies, then wave partials
    v = wave_sum_desc(v);
    const int tid = threadIdx.x;
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    float t = 0.0f;
    for (int w = 0; w < kWaves; ++w) t += red[w];
    return t;
}

// Three fixed-order workgroup sums with one pair of barriers; red: 3 x kWaves.
__device__ __forceinline__ void block_sum3_fixed(float &a, float &b, float &c, float *red)
{
    a = wave_sum_desc(a);
    b = wave_sum_desc(b);
    c = wave_sum_desc(c);
    const int tid = threadIdx.x;
    __syncthreads();
    if ((tid & 63) == 0) {
        red[tid >> 6] = a;
        red[kWaves + (tid >> 6)] = b;
        red[2 * kWaves + (tid >> 6)] = c;
    }
    __syncthreads();
    float ta = 0.0f, tb = 0.0f, tc = 0.0f;
    for (int w = 0; w < kWaves; ++w) {
        ta += red[w];
        tb += red[kWaves + w];
        tc += red[2 * kWaves + w];
    }
    a = ta;
    b = tb;
    c = tc;
}

// conv1 (1 -> 32 channels) on MFMA: the nine taps are the K dimension (padded
// to 32 with zeros), BF16 inputs and weights, FP32 accumulation, bias and
// ReLU in FP32; output [pixel][channel] BF16 as the other layers. As in the
// 32 -> 32 layers the weights are the A operand (16 output channels x 32
// taps) and the taps of 16 pixels the B operand, so each lane ends with four
// consecutive channels of one pixel and stores them with one 8-byte write.
// conv1's A operands (W1 with the taps as K, zero beyond tap 8) and its bias
// as this lane needs them. Loaded once per launch: read at every patch, the
// sixteen guarded loads each waited for their own round trip to L2.
typedef short s16x4 __attribute__((ext_vector_type(4)));  // four BF16 as the 16x16x16 MFMA takes them
struct Conv1W {
    s16x4 w0, w1;
    float b0[4], b1[4];
};
__device__ __forceinline__ Conv1W conv1_weights(const float *__restrict__ prm)
{
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    float v0[4], v1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {  // unconditional reads (tap clamped), so all are in flight together
        const int t = min(g * 4 + j, 8);
        v0[j] = prm[oW1 + t * kC + n];
        v1[j] = prm[oW1 + t * kC + 16 + n];
    }
    Conv1W c;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool tap = g * 4 + j < 9;
        c.w0[j] = __builtin_bit_cast(short, (__bf16)(tap ? v0[j] : 0.0f));
        c.w1[j] = __builtin_bit_cast(short, (__bf16)(tap ? v1[j] : 0.0f));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        c.b0[i] = prm[oB1 + g * 4 + i];
        c.b1[i] = prm[oB1 + 16 + g * 4 + i];
    }
    return c;
}

__device__ __forceinline__ void conv1_mfma(const float *__restrict__ xs, __bf16 *__restrict__ out,
                                           const Conv1W &cw, __bf16 *__restrict__ gout)
{
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = lane & 15, g = lane >> 4;  // n: output channel row of A / pixel of B; g: k-group
    const s16x4 w0 = cw.w0, w1 = cw.w1;
    const float *b0 = cw.b0, *b1 = cw.b1;
    // Every tile of this wave has the same column half (kWaves is even), so
    // the offset of tap j from the tile's row start, wrapped in x, is fixed
    // per lane; the row wrap is the wrap of the whole 1024-pixel plane.
    // Padded taps (t >= 9) read the centre pixel; their weights are zero.
    // K = 16 (the nine taps and zeros): four taps per lane.
    static_assert(kWaves % 2 == 0, "the column half of a wave's tiles must not change");
    const int x0 = (wave & 1) * 16;
    int off[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int t = g * 4 + j;
        const int tt = t < 9 ? t : 4;
        off[j] = tap_dy(tt) * kSide + wrap32(x0 + n + tap_dx(tt));  // rows -1 and 32 are xs's halo
    }
    // two tiles per iteration, all eight reads issued before either MFMA
    for (int tile = wave; tile < kPix / 16; tile += 2 * kWaves) {
        s16x4 a[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int ybase = ((tile + u * kWaves) >> 1) * kSide;
#pragma unroll
            for (int j = 0; j < 4; ++j) a[u][j] = __builtin_bit_cast(short, (__bf16)xs[ybase + off[j]]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const f32x4 z = {0.f, 0.f, 0.f, 0.f};
            const f32x4 acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w0, a[u], z, 0, 0, 0);
            const f32x4 acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1, a[u], z, 0, 0, 0);
            const int y = (tile + u * kWaves) >> 1;
            const int p = y * kSide + x0 + n;  // D column = pixel
            bf16x4 v0, v1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v0[i] = (__bf16)fmaxf(acc0[i] + b0[i], 0.0f);
                v1[i] = (__bf16)fmaxf(acc1[i] + b1[i], 0.0f);
            }
            *reinterpret_cast<bf16x4 *>(out + act_off(p, g >> 1) + (g & 1) * 4) = v0;
            *reinterpret_cast<bf16x4 *>(out + act_off(p, 2 + (g >> 1)) + (g & 1) * 4) = v1;
            if (y == 0 || y == kSide - 1) {  // the halo copy of the row (uniform over the wave)
                const int h = (y == 0 ? kSide : -kSide) * kActRow;
                *reinterpret_cast<bf16x4 *>(out + h + act_off(p, g >> 1) + (g & 1) * 4) = v0;
                *reinterpret_cast<bf16x4 *>(out + h + act_off(p, 2 + (g >> 1)) + (g & 1) * 4) = v1;
            }
            if (gout) {
                *reinterpret_cast<bf16x4 *>(gout + p * kC + g * 4) = v0;
                *reinterpret_cast<bf16x4 *>(gout + p * kC + 16 + g * 4) = v1;
            }
        }
    }
}

// BF16 copies of conv2..4 weights:
//   wf[l][tap][co][ci]  (forward B operand: 8 consecutive ci per lane)
//   wb[l][tap][ci][co]  (backward-data B operand: 8 consecutive co per lane)
__global__ void k_pack(const float *__restrict__ prm, __bf16 *__restrict__ wf, __bf16 *__restrict__ wb,
                       int *__restrict__ next)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *next = 0;  // patch counter of the following forward launch
    if (i >= 3 * 9 * kC * kC) return;
    const int l = i / (9 * kC * kC), r = i % (9 * kC * kC);
    const int tap = r / (kC * kC), ci = (r / kC) % kC, co = r % kC;
    const float w = prm[oW2 + l * (9 * kC * kC + kC) + r];  // W[tap][ci][co]
    wf[(size_t)l * 9 * kC * kC + (tap * kC + co) * kC + ci] = (__bf16)w;
    wb[(size_t)l * 9 * kC * kC + (tap * kC + ci) * kC + co] = (__bf16)w;
}

struct FwdArgs {
    const float *prm;
    const __bf16 *wf;       // [3][9][32][32]
    const float *logk;      // [B][1024]
    const int8_t *sym;      // [B] symmetry per patch (training) or null
    int n_sym;              // predictions averaged over symmetries 0..n_sym-1
    int batch;
    float *pred;            // [B][2] log kxx, log kyy
    float *stats;           // [B][8] mean, std, lag-1 corr x, y, the 4 features (or null)
    float *spread;          // [B][2] max - min over the n_sym predictions (or null)
    __bf16 *acts;           // [4][B][1024][32] when training, else null
    float *pool_out;        // [B][37] head input when training
    int *next;              // patches claimed beyond the first gridDim.x (zeroed by k_pack)
};

// One 3x3, 32 -> 32 layer on MFMA. in/out are [pixel][channel] BF16 in LDS
// (chunks permuted, act_off; halo rows). The product is D[co][pixel] =
// W[co][ci] X[ci][pixel] per tap (A: weights, held in registers; B: 8
// channels of one pixel per lane, one 16-byte LDS read), so each lane ends
// with 4 consecutive output channels of one pixel and stores them with one
// 8-byte write. Each wave takes eight 16-pixel tiles, the consecutive rows of
// one column half, reading each input row once for the three output rows it
// feeds (below). With POOL the ReLU outputs are summed per channel into
// pool_part[wave][32] instead of being stored.
// Address-space-qualified element types: a generic pointer makes the
// compiler emit flat memory instructions, which count against the LDS wait
// counter too, so every MFMA would wait for all LDS reads in flight.
typedef __attribute__((address_space(3))) __bf16 lds_bf16;     // LDS (32-bit addresses)
typedef __attribute__((address_space(1))) __bf16 glb_bf16;     // global memory
typedef __attribute__((address_space(1))) const float glb_f32;

// The packed BF16 weights of one 32 -> 32 layer (9 x 32 x 32) as 1152
// 16-byte chunks (row = tap * 32 + output channel, 4 chunks of 8 input
// channels per row); in LDS at act_off(row, chunk), the permutation of the
// activation buffers, so the 16 rows a wave reads per operand spread over
// the banks.
constexpr int kWChunks = 9 * kC * kC / 8;

template <bool POOL, bool PF, bool GOUT>
__device__ __forceinline__ void conv_body(const __bf16 *__restrict__ in_p, __bf16 *__restrict__ out_p,
                                          __bf16 *__restrict__ wbuf_p, const __bf16 *__restrict__ next_w,
                                          const float *__restrict__ bias, __bf16 *__restrict__ gout_p,
                                          float *__restrict__ pool_part, const float *__restrict__ pf, int pf_sym,
                                          float *__restrict__ xs_stage)
{
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) bf16x8 lds_bf16x8;
    typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;
    typedef __attribute__((address_space(1))) bf16x4 glb_bf16x4;
    typedef __attribute__((address_space(1))) const bf16x8 glb_bf16x8;
    const lds_bf16 *in = (const lds_bf16 *)in_p;
    lds_bf16 *out = (lds_bf16 *)out_p;
    glb_bf16 *gout = (glb_bf16 *)gout_p;
    lds_bf16 *wbuf = (lds_bf16 *)wbuf_p;
    const glb_bf16 *nw = (const glb_bf16 *)next_w;
    glb_f32 *bg = (glb_f32 *)bias;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = lane & 15, g = lane >> 4;  // n: pixel within the tile (B, D) / co row (A); g: k-group
    // Addressing: every tile of this wave has the same column half (kWaves is
    // even), and the chunk permutation of act_off depends on the column only,
    // so the column part of each tap's offset is fixed per lane (three
    // values, dx = -1, 0, 1) and a tap's LDS offset is a wave-uniform row
    // offset plus one of them.
    static_assert(kWaves % 2 == 0, "the column half of a wave's tiles must not change");
    const int x0 = (wave & 1) * 16;
    int colp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) colp[d] = act_off(wrap32(x0 + n + d - 1), g);
    const int col0 = x0 + n;
    const int op[2] = {act_off(col0, g >> 1) + (g & 1) * 4, act_off(col0, 2 + (g >> 1)) + (g & 1) * 4};
    // The bias is read from global memory first and waited for only where
    // it is used (a wait at each read cost one L2 round trip per layer).
    float bb[2][4];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) bb[ct][i] = bg[ct * 16 + g * 4 + i];
    // This layer's weights come from LDS, where the previous layer (or the
    // set-up before the first patch) staged them: every wave needs all of
    // them in registers, and eight waves reading 18 KB each through the
    // vector memory path cost about a third of the forward's time.
    bf16x8 w[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
            w[t][ct] = *reinterpret_cast<const lds_bf16x8 *>(wbuf + act_off(t * kC + ct * 16 + n, g));
    __syncthreads();
    // the bias has arrived meanwhile: with no register loads in flight, the
    // tiles wait for none of the loads below
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    // Once every wave holds its copy (the barrier), the next layer's weights
    // go from global memory straight into the same LDS buffer while this
    // layer's tiles run. A load to LDS writes lane l's bytes at the wave's
    // base + l x size, so each wave fills its own 2304 bytes of the buffer
    // with two 16-byte and one 4-byte load per lane, and each lane reads the
    // piece of the chunk whose permuted position (act_off) it fills. With PF
    // the next pass's input goes the same way into the input plane (free
    // once conv1 has run). Waited for at the end of the layer.
    typedef __attribute__((address_space(3))) void lds_void;
    typedef __attribute__((address_space(1))) const void glb_void;
    static_assert(kWChunks % kWaves == 0 && kWChunks / kWaves == 2 * 64 + 16, "three loads per wave");
    {
        typedef __attribute__((address_space(3))) char lds_char;
        lds_char *wb = (lds_char *)wbuf + wave * (kWChunks / kWaves) * 16;
        auto src = [&](int q, int dw) {  // dword dw of the chunk at permuted position q
            const int row = q >> 2, c = (q & 3) ^ ((row >> 1) & 3);
            return (glb_void *)(nw + row * kC + c * 8 + dw * 2);
        };
        const int q0 = wave * (kWChunks / kWaves);
        __builtin_amdgcn_global_load_lds(src(q0 + lane, 0), (lds_void *)wb, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(src(q0 + 64 + lane, 0), (lds_void *)(wb + 1024), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(src(q0 + 128 + (lane >> 2), lane & 3), (lds_void *)(wb + 2048), 4, 0, 0);
    }
    if (PF) {
        glb_f32 *pfg = (glb_f32 *)pf;
        __builtin_amdgcn_global_load_lds((glb_void *)(pfg + sym_src(threadIdx.x, pf_sym)),
                                         (lds_void *)(xs_stage + wave * 64), 4, 0, 0);
        __builtin_amdgcn_global_load_lds((glb_void *)(pfg + sym_src(threadIdx.x + kT, pf_sym)),
                                         (lds_void *)(xs_stage + kT + wave * 64), 4, 0, 0);
    }
    float ps[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    // The wave's tiles are the 8 consecutive rows r0 .. r0 + 7 (r0 = 8 x
    // (wave / 2)) of one column half. The input rows r0 - 1 .. r0 + 8 (halo
    // rows included) are read once each, three reads (dx = -1, 0, 1), and
    // each feeds the up to three output rows it is a tap row of, whose
    // accumulators roll through three slots: a third of the LDS reads of
    // reading nine operands per tile. Every tile still adds its taps in the
    // order t = 0..8. The epilogue of a row runs once its last tap row is in.
    const int r0 = (wave >> 1) * 8;
    const lds_bf16 *base[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) base[d] = in + r0 * kActRow + colp[d];
    lds_bf16 *obase = out + r0 * kActRow;
    constexpr int kRows = 8;
    f32x4 acc[3][2];
    auto epilogue = [&](int k, const f32x4 (&ac)[2]) {
        const int y = r0 + k;
        const int p = y * kSide + col0;  // D column = pixel
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            bf16x4 v;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float r = fmaxf(ac[ct][i] + bb[ct][i], 0.0f);
                if (POOL) ps[ct][i] += r;
                v[i] = (__bf16)r;
            }
            if (!POOL) {
                *reinterpret_cast<lds_bf16x4 *>(obase + k * kActRow + op[ct]) = v;
                // rows 0 and 31 also go to their halo copies (uniform over the wave)
                if (k == 0 && r0 == 0) *reinterpret_cast<lds_bf16x4 *>(obase + kSide * kActRow + op[ct]) = v;
                if (k == kRows - 1 && r0 == kSide - kRows)
                    *reinterpret_cast<lds_bf16x4 *>(obase + (k - kSide) * kActRow + op[ct]) = v;
            }
            if (GOUT) *reinterpret_cast<glb_bf16x4 *>(gout + p * kC + ct * 16 + g * 4) = v;
        }
    };
    bf16x8 x[2][3];  // the operands of input rows i and i + 1
#pragma unroll
    for (int d = 0; d < 3; ++d) x[0][d] = *reinterpret_cast<const lds_bf16x8 *>(base[d] - kActRow);
#pragma unroll
    for (int i = 0; i < kRows + 2; ++i) {  // input row r0 - 1 + i
        const int cur = i & 1;
        // one row ahead only (hoisting every read to the top would need
        // registers for all of them)
        __builtin_amdgcn_sched_barrier(0);
        if (i + 1 < kRows + 2) {
#pragma unroll
            for (int d = 0; d < 3; ++d)
                x[cur ^ 1][d] = *reinterpret_cast<const lds_bf16x8 *>(base[d] + i * kActRow);
        }
        // output rows k = i (tap row dy = -1), i - 1 (dy = 0), i - 2 (dy = 1)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const int k = i - 1 - dy;
            if (k < 0 || k >= kRows) continue;
            f32x4 (&ac)[2] = acc[k % 3];
            if (dy == -1) ac[0] = ac[1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int t = 3 * (dy + 1) + d;
                ac[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[t][0], x[cur][d], ac[0], 0, 0, 0);
                ac[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[t][1], x[cur][d], ac[1], 0, 0, 0);
            }
            if (dy == 1) epilogue(k, ac);
        }
    }
    // the loads to LDS above have landed before the caller's barrier
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    if (POOL) {
        // lanes n = 0..15 of a k-group hold the same 4 channels for different
        // pixels: fixed-order butterfly over n
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = group_sum16(ps[ct][i]);
                if (n == 0) pool_part[wave * kC + ct * 16 + g * 4 + i] = v;
            }
    }
}

// The layer as the kernel inlines it. Its body comes from a function with
// restrict-qualified pointers, so its memory accesses carry alias scopes:
// with them the compiler can tell that the layer's LDS reads do not touch
// what the loads to LDS are writing, and does not wait for those loads first.
// (As a call, the layer paid a full wait at entry and register saves.)
template <bool POOL, bool PF, bool GOUT>
__device__ __forceinline__ void conv_mfma(const __bf16 *in_p, __bf16 *out_p, __bf16 *wbuf_p, const __bf16 *next_w,
                                          const float *bias, __bf16 *gout_p, float *pool_part, const float *pf,
                                          int pf_sym, float *xs_stage)
{
    conv_body<POOL, PF, GOUT>(in_p, out_p, wbuf_p, next_w, bias, gout_p, pool_part, pf, pf_sym, xs_stage);
}

// TRAIN: the activations stored for the backward pass (a.acts) and, when
// a.sym is given, a symmetry per patch from it rather than symmetries
// 0 .. n_sym - 1; the inference build reads and writes nothing else per pass.
template <bool TRAIN>
__global__ __launch_bounds__(kT) void k_forward(FwdArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16 *bufA = reinterpret_cast<__bf16 *>(smem) + kActRow;  // row 0 of a buffer with halo rows
    __bf16 *bufB = bufA + kActElems;
    float *xs = reinterpret_cast<float *>(bufB - kActRow + kActElems) + kSide;  // [1024], halo rows around it
    float *pool_part = xs + kPix + kSide;                     // [8][32]
    float *red = pool_part + kWaves * kC;                      // [8]
    float *head = red + kWaves;                                // [37]
    float *tmp = head + kZ + 3;                                // [16]
    float *red3 = tmp + 16;                                    // [3][8]
    __bf16 *wbuf = reinterpret_cast<__bf16 *>(red3 + 3 * kWaves);  // staged conv weights [1152 x 8]
    const int tid = threadIdx.x;
    const float *prm = a.prm;

    // Patches are claimed one at a time (each workgroup starts with its own
    // index, then takes the next free one), so workgroups that start late --
    // behind other work on the device -- simply take fewer patches. A
    // workgroup claims its next patch when it starts a patch and reads the
    // next pass's input during conv2 of the current one, so neither the
    // atomic nor the input read waits in line with the layers.
    __shared__ int claimed;
    // The patch mean and its four series/parallel features do not depend on
    // the symmetry a pass applies (a transposition exchanges the row and
    // column features): passes after the first take them from here.
    __shared__ float pass0[5];
    // conv2's weights into LDS before the first patch; each conv layer then
    // stages the next one's (conv4 stages conv2's for the next pass)
    for (int i = tid; i < kWChunks; i += kT)
        *reinterpret_cast<bf16x8 *>(wbuf + act_off(i >> 2, i & 3)) =
            *reinterpret_cast<const bf16x8 *>(a.wf + (i >> 2) * kC + (i & 3) * 8);
    // the first pass's input, staged where conv2 stages the later ones (each
    // thread reads back only what it wrote)
    if (blockIdx.x < a.batch) {
        const int s0 = TRAIN && a.sym ? (int)a.sym[blockIdx.x] : 0;
        const float *lk0 = a.logk + (size_t)blockIdx.x * kPix;
        xs[tid] = lk0[sym_src(tid, s0)];
        xs[tid + kT] = lk0[sym_src(tid + kT, s0)];
    }
    // launch constants in registers: conv1's operands and the head's weights
    // for this thread (hidden unit h = tid / 16 and inputs j, j + 16, j + 32)
    const Conv1W c1w = conv1_weights(prm);
    const int hh = tid >> 4, hj = tid & 15;
    const float m1a = prm[oM1 + hh * kZ + hj], m1b = prm[oM1 + hh * kZ + hj + 16];
    const float m1c = hj + 32 < kZ ? prm[oM1 + hh * kZ + min(hj + 32, kZ - 1)] : 0.0f;
    const float c1h = prm[oC1 + hh], m2a = prm[oM2 + hh], m2b = prm[oM2 + kH + hh];
    const float c2a = prm[oC2], c2b = prm[oC2 + 1];
    __syncthreads();
    for (int b = blockIdx.x; b < a.batch;) {
        float acc0 = 0.0f, acc1 = 0.0f;  // averaged prediction (thread 0)
        float lo0 = INFINITY, hi0 = -INFINITY, lo1 = INFINITY, hi1 = -INFINITY;  // their range
        for (int t = 0; t < a.n_sym; ++t) {
            const int sym = TRAIN && a.sym ? (int)a.sym[b] : t;
            // the next patch, claimed now and used after conv1; a wrapping
            // increment (no wrap below 2^32 - 1), since the compiler's
            // wave-level rewrite of an add would wait for the result at once
            int nxt;
            if (tid == 0 && t == 0) nxt = (int)atomicInc(reinterpret_cast<unsigned *>(a.next), 0xffffffffu);
            // ---- input under the symmetry (staged), centring (FP32) ----
            const float v0 = xs[tid], v1 = xs[tid + kT];
            const float m = t == 0 ? block_sum_fixed(v0 + v1, red) * (1.0f / kPix) : pass0[0];
            const float x0 = v0 - m, x1 = v1 - m;
            xs[tid] = x0;
            xs[tid + kT] = x1;
            if (tid < kSide) xs[kPix + tid] = x0;                // row 32 = row 0
            if (tid >= kT - kSide) xs[tid + kT - kPix] = x1;    // row -1 = row 31
            __syncthreads();
            if (a.stats && t == 0) {
                // variance and lag-1 correlations of the centred field (periodic)
                const int p0 = tid, p1 = tid + kT;
                const float rx = x0 * xs[(p0 & ~31) | wrap32(p0 + 1)] + x1 * xs[(p1 & ~31) | wrap32(p1 + 1)];
                const float ry = x0 * xs[(p0 + kSide) & (kPix - 1)] + x1 * xs[(p1 + kSide) & (kPix - 1)];
                float var = x0 * x0 + x1 * x1, cx = rx, cy = ry;
                block_sum3_fixed(var, cx, cy, red3);
                var *= 1.0f / kPix;
                cx *= 1.0f / kPix;
                cy *= 1.0f / kPix;
                if (tid == 0) {
                    float *st = a.stats + 8 * (size_t)b;
                    st[0] = m;
                    st[1] = sqrtf(var);
                    st[2] = var > 0.f ? cx / var : 0.f;
                    st[3] = var > 0.f ? cy / var : 0.f;
                }
            }
            if (t == 0) {
                series_parallel(xs, tmp, head + kC + 1);
                if (a.stats && tid < 4) a.stats[8 * (size_t)b + 4 + tid] = head[kC + 1 + tid];
                if (tid < 5) pass0[tid] = tid == 0 ? m : head[kC + tid];
            } else if (tid < 4) {
                // features 0, 1 along rows and columns, 2, 3 along columns and rows
                head[kC + 1 + tid] = pass0[1 + ((sym & 1) ? tid ^ 2 : tid)];
            }
            // ---- conv1: 1 -> 32 channels on MFMA ----
            __bf16 *g1 = TRAIN ? a.acts + ((size_t)0 * a.batch + b) * kPix * kC : nullptr;
            conv1_mfma(xs, bufA, c1w, g1);
            if (tid == 0 && t == 0) claimed = (int)gridDim.x + nxt;
            __syncthreads();
            // the next pass: this patch under the next symmetry, or the
            // claimed patch (none past the batch)
            const int bn = t + 1 < a.n_sym ? b : claimed;
            const bool more = bn < a.batch;
            // with no next pass, the current patch is read again and not used
            const float *pf = a.logk + (size_t)(more ? bn : b) * kPix;
            const int sn = t + 1 < a.n_sym ? (TRAIN && a.sym ? sym : t + 1)
                                           : (TRAIN && a.sym && more ? (int)a.sym[bn] : 0);
            // ---- conv2..conv4 on MFMA ----
            __bf16 *g2 = TRAIN ? a.acts + ((size_t)1 * a.batch + b) * kPix * kC : nullptr;
            __bf16 *g3 = TRAIN ? a.acts + ((size_t)2 * a.batch + b) * kPix * kC : nullptr;
            __bf16 *g4 = TRAIN ? a.acts + ((size_t)3 * a.batch + b) * kPix * kC : nullptr;
            conv_mfma<false, true, TRAIN>(bufA, bufB, wbuf, a.wf + 9 * kC * kC, prm + oB2, g2, pool_part, pf, sn,
                                          xs);
            __syncthreads();
            conv_mfma<false, false, TRAIN>(bufB, bufA, wbuf, a.wf + 2 * 9 * kC * kC, prm + oB3, g3, pool_part,
                                           nullptr, 0, nullptr);
            __syncthreads();
            // stages conv2's weights for the next pass
            conv_mfma<true, false, TRAIN>(bufA, nullptr, wbuf, a.wf, prm + oB4, g4, pool_part, nullptr, 0, nullptr);
            __syncthreads();
            // ---- pooling and head (FP32) ----
            if (tid < kC) {
                float sp = 0.0f;
                for (int w = 0; w < kWaves; ++w) sp += pool_part[w * kC + tid];
                head[tid] = sp * (1.0f / kPix);
            }
            if (tid == 0) head[kC] = m;
            __syncthreads();
            {
                // hidden unit h on 16 threads, each summing inputs k = j, j + 16, j + 32
                const int j = hj;
                float zh = 0.0f;
                zh += m1a * head[j];
                zh += m1b * head[j + 16];
                if (j + 32 < kZ) zh += m1c * head[j + 32];
                zh = group_sum16(zh);
                const float hval = fmaxf(zh + c1h, 0.0f);
                // the first lane of each 16-lane row holds its unit's terms
                const float y0 = rows_sum_lane0(j == 0 ? m2a * hval : 0.0f);
                const float y1 = rows_sum_lane0(j == 0 ? m2b * hval : 0.0f);
                if ((tid & 63) == 0) {
                    red3[tid >> 6] = y0;
                    red3[kWaves + (tid >> 6)] = y1;
                }
                if (a.pool_out && tid < kZ) a.pool_out[(size_t)b * kZ + tid] = head[tid];
                __syncthreads();
                if (tid == 0) {
                    float s0 = 0.0f, s1 = 0.0f;
                    for (int w = 0; w < kWaves; ++w) {
                        s0 += red3[w];
                        s1 += red3[kWaves + w];
                    }
                    s0 += c2a + m;
                    s1 += c2b + m;
                    // a transposed patch predicts (kyy, kxx) of the original
                    const float q0 = (sym & 1) ? s1 : s0, q1 = (sym & 1) ? s0 : s1;
                    acc0 += q0;
                    acc1 += q1;
                    lo0 = fminf(lo0, q0);
                    hi0 = fmaxf(hi0, q0);
                    lo1 = fminf(lo1, q1);
                    hi1 = fmaxf(hi1, q1);
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            a.pred[2 * (size_t)b] = acc0 / a.n_sym;
            a.pred[2 * (size_t)b + 1] = acc1 / a.n_sym;
            if (a.spread) {
                a.spread[2 * (size_t)b] = hi0 - lo0;
                a.spread[2 * (size_t)b + 1] = hi1 - lo1;
            }
        }
        // written after conv1 of this patch's first pass; the next write
        // comes after the barriers of the next patch's first pass
        b = claimed;
    }
}

// Statistics of each patch only (the range detector's inputs), computed
// exactly as k_forward computes them for its d_stats output.
__global__ __launch_bounds__(kT) void k_stats(const float *__restrict__ logk, int batch,
                                              float *__restrict__ stats)
{
    __shared__ float xs[kPix];
    __shared__ float red[kWaves];
    __shared__ float red3[3 * kWaves];
    __shared__ float tmp[128];
    __shared__ float feat[4];
    const int tid = threadIdx.x;
    for (int b = blockIdx.x; b < batch; b += gridDim.x) {
        const float *lk = logk + (size_t)b * kPix;
        const float v0 = lk[tid], v1 = lk[tid + kT];
        const float m = block_sum_fixed(v0 + v1, red) * (1.0f / kPix);
        const float x0 = v0 - m, x1 = v1 - m;
        xs[tid] = x0;
        xs[tid + kT] = x1;
        __syncthreads();
        const int p0 = tid, p1 = tid + kT;
        const float rx = x0 * xs[(p0 & ~31) | wrap32(p0 + 1)] + x1 * xs[(p1 & ~31) | wrap32(p1 + 1)];
        const float ry = x0 * xs[(p0 + kSide) & (kPix - 1)] + x1 * xs[(p1 + kSide) & (kPix - 1)];
        float var = x0 * x0 + x1 * x1, cx = rx, cy = ry;
        block_sum3_fixed(var, cx, cy, red3);
        var *= 1.0f / kPix;
        cx *= 1.0f / kPix;
        cy *= 1.0f / kPix;
        series_parallel(xs, tmp, feat);
        if (tid == 0) {
            float *st = stats + 8 * (size_t)b;
            st[0] = m;
            st[1] = sqrtf(var);
            st[2] = var > 0.f ? cx / var : 0.f;
            st[3] = var > 0.f ? cy / var : 0.f;
        }
        if (tid < 4) stats[8 * (size_t)b + 4 + tid] = feat[tid];
        __syncthreads();
    }
}

// Head backward per patch (one wave per patch), FP32. Loss L = mean over the
// batch and both outputs of (prediction - target)^2. Writes the patch's head
// gradient, dL/dpool and its loss term.
__global__ __launch_bounds__(64) void k_head_backward(const float *__restrict__ prm,
                                                      const float *__restrict__ pool, const float *__restrict__ target,
                                                      const int8_t *__restrict__ sym, int batch,
                                                      float *__restrict__ ghead, float *__restrict__ dpool,
                                                      float *__restrict__ loss_terms)
{
    const int b = blockIdx.x, j = threadIdx.x;
    if (b >= batch) return;
    __shared__ float z[kZ], dh[kH], hh[kH];
    __shared__ float dyv[2];
    if (j < kZ) z[j] = pool[(size_t)b * kZ + j];
    __syncthreads();
    float hpre = 0.0f, h = 0.0f;
    if (j < kH) {
        hpre = prm[oC1 + j];
        for (int k = 0; k < kZ; ++k) hpre += prm[oM1 + j * kZ + k] * z[k];
        h = fmaxf(hpre, 0.0f);
        hh[j] = h;
    }
    float y0 = j < kH ? prm[oM2 + j] * h : 0.0f, y1 = j < kH ? prm[oM2 + kH + j] * h : 0.0f;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        y0 += __shfl_xor(y0, off, 64);
        y1 += __shfl_xor(y1, off, 64);
    }
    const float m = z[kC];
    // a transposed patch is trained on the exchanged targets
    const int tr = (sym && (sym[b] & 1)) ? 1 : 0;
    const float e0 = y0 + prm[oC2] + m - target[2 * (size_t)b + tr];
    const float e1 = y1 + prm[oC2 + 1] + m - target[2 * (size_t)b + 1 - tr];
    const float scale = 2.0f / (2.0f * batch);
    if (j == 0) {
        dyv[0] = scale * e0;
        dyv[1] = scale * e1;
        loss_terms[b] = (e0 * e0 + e1 * e1) / (2.0f * batch);
    }
    __syncthreads();
    float *g = ghead + (size_t)b * kNHead;  // same order as the parameters from oM1
    if (j < kH) {
        g[(oM2 - oM1) + j] = dyv[0] * hh[j];
        g[(oM2 - oM1) + kH + j] = dyv[1] * hh[j];
        const float d = (hpre > 0.0f) ? (dyv[0] * prm[oM2 + j] + dyv[1] * prm[oM2 + kH + j]) : 0.0f;
        dh[j] = d;
        g[(oC1 - oM1) + j] = d;
        for (int k = 0; k < kZ; ++k) g[j * kZ + k] = d * z[k];
    }
    if (j < 2) g[(oC2 - oM1) + j] = dyv[j];
    __syncthreads();
    if (j < kC) {
        float s = 0.0f;
        for (int k = 0; k < kH; ++k) s += dh[k] * prm[oM1 + k * kZ + j];
        dpool[(size_t)b * kC + j] = s;
    }
}

struct BwdArgs {
    const float *prm;
    const __bf16 *wb;      // [3][9][ci][co]
    const float *logk;     // [B][1024]
    const int8_t *sym;     // [B] or null
    const __bf16 *acts;    // [4][B][1024][32]
    const float *dpool;    // [B][32]
    int batch;
    float *gpart;          // [gridDim.x][kNConv] per-workgroup partial conv gradients
};

// dW for one 32 -> 32 layer: wave w owns tile-jobs j = w, w + 8, ... of the
// 36 (tap, co-tile, ci-tile) jobs; each job is a 16 x 16 block of dW[tap]
// accumulated over the 1024 pixels (K) with D[m = co][n = ci].
__device__ __forceinline__ void dw_mfma(const __bf16 *__restrict__ X, const __bf16 *__restrict__ dZ, f32x4 acc[5])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    int jj = 0;
    for (int job = wave; job < 36; job += kWaves, ++jj) {
        const int tap = job >> 2, cot = (job >> 1) & 1, cit = job & 1;
        const int dy = tap_dy(tap), dx = tap_dx(tap);
        f32x4 c = acc[jj];
        for (int k0 = 0; k0 < kPix; k0 += 32) {
            bf16x8 av, bv;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int p = k0 + g * 8 + i;  // pixel (K index)
                av[i] = dZ[p * kC + cot * 16 + n];                       // A[m = co][k = p]
                const int q = wrap32((p >> 5) + dy) * kSide + wrap32((p & 31) + dx);
                bv[i] = X[q * kC + cit * 16 + n];                        // B[k = p][n = ci]
            }
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
        }
        acc[jj] = c;
    }
}

// dX = conv-transpose(dZ, W), times the ReLU mask of X, written over X.
__device__ __forceinline__ void dx_mfma(__bf16 *__restrict__ X, const __bf16 *__restrict__ dZ,
                                        const __bf16 *__restrict__ wbl)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    bf16x8 w[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)  // n indexes ci within tile ct; 8 consecutive co per lane
            w[t][ct] = *reinterpret_cast<const bf16x8 *>(wbl + (t * kC + ct * 16 + n) * kC + g * 8);
    for (int tile = wave; tile < kPix / 16; tile += kWaves) {
        const int y = tile >> 1, x0 = (tile & 1) * 16;
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            // out[p] uses in[p + tap]: the gradient at p comes from dZ[p - tap]
            const int p = wrap32(y - tap_dy(t)) * kSide + wrap32(x0 + n - tap_dx(t));
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(dZ + p * kC + g * 8);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, w[t][0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, w[t][1], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int p = y * kSide + x0 + g * 4 + i;
            const float m0 = (float)X[p * kC + n] > 0.0f ? 1.0f : 0.0f;
            const float m1 = (float)X[p * kC + 16 + n] > 0.0f ? 1.0f : 0.0f;
            X[p * kC + n] = (__bf16)(acc0[i] * m0);
            X[p * kC + 16 + n] = (__bf16)(acc1[i] * m1);
        }
    }
}

__device__ __forceinline__ void load_act(__bf16 *__restrict__ dst, const __bf16 *__restrict__ src)
{
    const bf16x8 *s = reinterpret_cast<const bf16x8 *>(src);
    bf16x8 *d = reinterpret_cast<bf16x8 *>(dst);
    for (int i = threadIdx.x; i < kPix * kC / 8; i += kT) d[i] = s[i];
}

__global__ __launch_bounds__(kT) void k_backward(BwdArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16 *buf0 = reinterpret_cast<__bf16 *>(smem);
    __bf16 *buf1 = buf0 + kPix * kC;
    float *xs = reinterpret_cast<float *>(buf1 + kPix * kC);  // [1024]
    float *red = xs + kPix;                                   // [8]
    float *dz1 = red + kWaves;                                // [32] scratch for bias grads
    const int tid = threadIdx.x;
    f32x4 acc[3][5];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int j = 0; j < 5; ++j) acc[l][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // conv1 weight/bias and conv2..4 bias gradients: thread tid owns entries
    float gw1[1] = {0.0f};  // W1[tap][co] entry tid (tid < 288)
    float gb[4] = {0.f, 0.f, 0.f, 0.f};  // bias of layer l for channel tid (tid < 32)

    for (int b = blockIdx.x; b < a.batch; b += gridDim.x) {
        const size_t stride = (size_t)a.batch * kPix * kC;
        const __bf16 *act = a.acts + (size_t)b * kPix * kC;
        // dZ4 = dpool / 1024 where a4 > 0 (a4 from the forward)
        load_act(buf0, act + 3 * stride);
        __syncthreads();
        for (int i = tid; i < kPix * kC; i += kT) {
            const float d = a.dpool[(size_t)b * kC + (i & 31)] * (1.0f / kPix);
            buf0[i] = (__bf16)((float)buf0[i] > 0.0f ? d : 0.0f);
        }
        __bf16 *dZ = buf0, *X = buf1;
        for (int l = 3; l >= 1; --l) {  // layer l + 1 of the network: conv2..4 are l = 1..3
            load_act(X, act + (size_t)(l - 1) * stride);
            __syncthreads();
            // bias gradient of this layer: sum over pixels of dZ
            if (tid < kC) {
                float s = 0.0f;
                for (int p = 0; p < kPix; ++p) s += (float)dZ[p * kC + tid];
                gb[l] += s;
            }
            dw_mfma(X, dZ, acc[l - 1]);
            __syncthreads();
            dx_mfma(X, dZ, a.wb + (size_t)(l - 1) * 9 * kC * kC);
            __syncthreads();
            __bf16 *t = dZ;
            dZ = X;
            X = t;
        }
        // layer 1 (1 -> 32), FP32: x from the input
        const float *lk = a.logk + (size_t)b * kPix;
        const int sym = a.sym ? (int)a.sym[b] : 0;
        const float v0 = lk[sym_src(tid, sym)], v1 = lk[sym_src(tid + kT, sym)];
        const float m = block_sum_fixed(v0 + v1, red) * (1.0f / kPix);
        xs[tid] = v0 - m;
        xs[tid + kT] = v1 - m;
        __syncthreads();
        if (tid < kC) {
            float s = 0.0f;
            for (int p = 0; p < kPix; ++p) s += (float)dZ[p * kC + tid];
            gb[0] += s;
        }
        if (tid < 9 * kC) {
            const int tap = tid / kC, co = tid % kC;
            const int dy = tap_dy(tap), dx = tap_dx(tap);
            float s = 0.0f;
            for (int p = 0; p < kPix; ++p) {
                const int q = wrap32((p >> 5) + dy) * kSide + wrap32((p & 31) + dx);
                s += xs[q] * (float)dZ[p * kC + co];
            }
            gw1[0] += s;
        }
        __syncthreads();
    }
    (void)dz1;
    // write this workgroup's partial conv gradients
    float *gp = a.gpart + (size_t)blockIdx.x * kNConv;
    if (tid < 9 * kC) gp[oW1 + tid] = gw1[0];
    if (tid < kC) {
        gp[oB1 + tid] = gb[0];
        gp[oB2 + tid] = gb[1];
        gp[oB3 + tid] = gb[2];
        gp[oB4 + tid] = gb[3];
    }
    const int lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        float *gw = gp + oW2 + l * (9 * kC * kC + kC);  // W[tap][ci][co]
        int jj = 0;
        for (int job = wave; job < 36; job += kWaves, ++jj) {
            const int tap = job >> 2, cot = (job >> 1) & 1, cit = job & 1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = cot * 16 + g * 4 + i;  // D row m = co
                const int ci = cit * 16 + n;          // D col n = ci
                gw[(tap * kC + ci) * kC + co] = acc[l][jj][i];
            }
        }
    }
}

// grad = sum over workgroups of the conv partials (fixed order), and the sum
// over patches of the head gradients; loss = sum of the loss terms.
__global__ void k_reduce(const float *__restrict__ gpart, int nparts, const float *__restrict__ ghead, int batch,
                         const float *__restrict__ loss_terms, float *__restrict__ grad, float *__restrict__ loss)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNConv) {
        float s = 0.0f;
        for (int w = 0; w < nparts; ++w) s += gpart[(size_t)w * kNConv + i];
        grad[i] = s;
    } else if (i < kNParams) {
        const int j = i - kNConv;
        float s = 0.0f;
        for (int b = 0; b < batch; ++b) s += ghead[(size_t)b * kNHead + j];
        grad[i] = s;
    } else if (i == kNParams) {
        float s = 0.0f;
        for (int b = 0; b < batch; ++b) s += loss_terms[b];
        *loss = s;
    }
}

__global__ void k_adam(float *__restrict__ prm, float *__restrict__ mom, float *__restrict__ vel,
                       const float *__restrict__ grad, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    const float g = grad[i];
    const float m = b1 * mom[i] + (1.0f - b1) * g;
    const float v = b2 * vel[i] + (1.0f - b2) * g * g;
    mom[i] = m;
    vel[i] = v;
    prm[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

struct SurLayout {
    size_t off_wf, off_wb, off_next, off_acts, off_pool, off_dpool, off_ghead, off_loss_terms, off_gpart,
        off_grad, off_loss, off_pred, total;
    int grid;
};

SurLayout sur_layout(int batch, bool train)
{
    SurLayout L{};
    L.grid = std::max(1, std::min(batch, 256));
    const size_t B = std::max(batch, 1);
    size_t off = 0;
    L.off_wf = off; off = align_up(off + 3 * 9 * kC * kC * 2);
    L.off_wb = off; off = align_up(off + 3 * 9 * kC * kC * 2);
    L.off_next = off; off = align_up(off + sizeof(int));
    if (train) {
        L.off_acts = off;       off = align_up(off + 4 * B * kPix * kC * 2);
        L.off_pool = off;       off = align_up(off + B * kZ * 4);
        L.off_dpool = off;      off = align_up(off + B * kC * 4);
        L.off_ghead = off;      off = align_up(off + B * kNHead * 4);
        L.off_loss_terms = off; off = align_up(off + B * 4);
        L.off_gpart = off;      off = align_up(off + (size_t)L.grid * kNConv * 4);
        L.off_grad = off;       off = align_up(off + kNParams * 4);
        L.off_loss = off;       off = align_up(off + 4);
        L.off_pred = off;       off = align_up(off + B * 2 * 4);
    }
    L.total = off;
    return L;
}

constexpr size_t kFwdLds = 2 * kActElems * 2 + (kPix + 2 * kSide + kWaves * kC + kWaves + kZ + 3 + 16 + 3 * kWaves) * 4 +
                           kWChunks * 16;
static_assert((2 * kActElems * 2 + (kPix + 2 * kSide + kWaves * kC + kWaves + kZ + 3 + 16 + 3 * kWaves) * 4) % 16 == 0,
              "the staged weights need 16-byte alignment");
static_assert(kFwdLds + 64 <= 160 * 1024, "forward LDS exceeds a CU's 160 KB");
constexpr size_t kBwdLds = 2 * kPix * kC * 2 + (kPix + kWaves + kC) * 4;

lbm_status check_ws(void *d_ws, size_t ws_bytes, size_t need, const char *fn)
{
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0 || ws_bytes < need)
        return set_error(LBM_EWORKSPACE, std::string(fn) + ": workspace NULL, misaligned or smaller than " +
                                             std::to_string(need));
    return LBM_OK;
}

lbm_status pack(const float *prm, char *ws, const SurLayout &L, hipStream_t stream)
{
    const int n = 3 * 9 * kC * kC;
    hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, stream, prm,
                       reinterpret_cast<__bf16 *>(ws + L.off_wf), reinterpret_cast<__bf16 *>(ws + L.off_wb),
                       reinterpret_cast<int *>(ws + L.off_next));
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

lbm_status forward(const float *prm, int batch, const float *logk, const int8_t *sym, int n_sym, float *pred,
                   float *stats, char *ws, const SurLayout &L, bool train, hipStream_t stream,
                   int max_workgroups = 0, float *spread = nullptr)
{
    FwdArgs a{};
    a.spread = spread;
    a.prm = prm;
    a.wf = reinterpret_cast<const __bf16 *>(ws + L.off_wf);
    a.logk = logk;
    a.sym = sym;
    a.n_sym = sym ? 1 : n_sym;
    a.batch = batch;
    a.pred = pred;
    a.stats = stats;
    a.acts = train ? reinterpret_cast<__bf16 *>(ws + L.off_acts) : nullptr;
    a.pool_out = train ? reinterpret_cast<float *>(ws + L.off_pool) : nullptr;
    a.next = reinterpret_cast<int *>(ws + L.off_next);
    LBM_HIP(hipFuncSetAttribute((const void *)k_forward<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kFwdLds));
    LBM_HIP(hipFuncSetAttribute((const void *)k_forward<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kFwdLds));
    const int cap = max_workgroups > 0 ? std::min(max_workgroups, device_cu_count()) : device_cu_count();
    const int grid = std::max(1, std::min(batch, cap));
    if (train)
        hipLaunchKernelGGL(k_forward<true>, dim3(grid), dim3(kT), kFwdLds, stream, a);
    else
        hipLaunchKernelGGL(k_forward<false>, dim3(grid), dim3(kT), kFwdLds, stream, a);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

lbm_status gradients(const float *prm, int batch, const float *logk, const int8_t *sym, const float *target,
                     float *pred, char *ws, const SurLayout &L, hipStream_t stream)
{
    lbm_status s = pack(prm, ws, L, stream);
    if (s != LBM_OK) return s;
    s = forward(prm, batch, logk, sym, 1, pred, nullptr, ws, L, true, stream);
    if (s != LBM_OK) return s;
    float *pool = reinterpret_cast<float *>(ws + L.off_pool);
    float *dpool = reinterpret_cast<float *>(ws + L.off_dpool);
    float *ghead = reinterpret_cast<float *>(ws + L.off_ghead);
    float *lterms = reinterpret_cast<float *>(ws + L.off_loss_terms);
    hipLaunchKernelGGL(k_head_backward, dim3(batch), dim3(64), 0, stream, prm, pool, target, sym, batch, ghead,
                       dpool, lterms);
    LBM_HIP(hipGetLastError());
    BwdArgs b{};
    b.prm = prm;
    b.wb = reinterpret_cast<const __bf16 *>(ws + L.off_wb);
    b.logk = logk;
    b.sym = sym;
    b.acts = reinterpret_cast<const __bf16 *>(ws + L.off_acts);
    b.dpool = dpool;
    b.batch = batch;
    b.gpart = reinterpret_cast<float *>(ws + L.off_gpart);
    LBM_HIP(hipFuncSetAttribute((const void *)k_backward, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBwdLds));
    hipLaunchKernelGGL(k_backward, dim3(L.grid), dim3(kT), kBwdLds, stream, b);
    LBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3((kNParams + 1 + 255) / 256), dim3(256), 0, stream,
                       reinterpret_cast<const float *>(ws + L.off_gpart), L.grid, ghead, batch, lterms,
                       reinterpret_cast<float *>(ws + L.off_grad), reinterpret_cast<float *>(ws + L.off_loss));
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" int32_t lbm_cnn_param_count(void) { return kNParams; }

extern "C" lbm_status lbm_patch_stats(int32_t batch, const float *d_logk, float *d_stats, hipStream_t stream)
{
    if (batch < 1 || !d_logk || !d_stats)
        return set_error(LBM_EINVAL, "lbm_patch_stats: batch < 1 or NULL argument");
    const int grid = std::min(batch, 8 * device_cu_count());
    hipLaunchKernelGGL(k_stats, dim3(grid), dim3(kT), 0, stream, d_logk, batch, d_stats);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" size_t lbm_cnn_workspace_bytes(int32_t batch, int32_t training)
{
    if (batch < 1) return 0;
    return sur_layout(batch, training != 0).total;
}

extern "C" lbm_status lbm_cnn_forward_limited(const float *d_params, int32_t batch, const float *d_logk,
                                              int32_t n_sym, float *d_pred, float *d_stats,
                                              int32_t max_workgroups, void *d_ws, size_t ws_bytes,
                                              hipStream_t stream)
{
    if (batch < 1 || !d_params || !d_logk || !d_pred)
        return set_error(LBM_EINVAL, "lbm_cnn_forward: batch < 1 or NULL argument");
    if (n_sym < 1 || n_sym > 8) return set_error(LBM_EINVAL, "lbm_cnn_forward: n_sym must lie in [1, 8]");
    if (max_workgroups < 0) return set_error(LBM_EINVAL, "lbm_cnn_forward: max_workgroups must be >= 0");
    const SurLayout L = sur_layout(batch, false);
    lbm_status s = check_ws(d_ws, ws_bytes, L.total, "lbm_cnn_forward");
    if (s != LBM_OK) return s;
    char *ws = static_cast<char *>(d_ws);
    s = pack(d_params, ws, L, stream);
    if (s != LBM_OK) return s;
    return forward(d_params, batch, d_logk, nullptr, n_sym, d_pred, d_stats, ws, L, false, stream,
                   max_workgroups);
}

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};

// Device address of `scratch` on the current device, looked up on the first
// call on that device (with it current) and kept.
lbm_status scratch_address(void **out)
{
    int dev = -1;
    LBM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(LBM_EDEVICE, "lbm_cnn_forward_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_check(e, "lbm_cnn_forward_noalloc: hipGetSymbolAddress(scratch)");
        if (!p) return set_error(LBM_EDEVICE, "lbm_cnn_forward_noalloc: scratch has no device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}
}  // namespace

extern "C" lbm_status lbm_cnn_forward_noalloc(const float *d_params, int32_t batch, const float *d_logk,
                                              int32_t n_sym, float *d_pred, float *d_stats,
                                              int32_t max_workgroups, hipStream_t stream)
{
    if (batch < 1 || !d_params || !d_logk || !d_pred)
        return set_error(LBM_EINVAL, "lbm_cnn_forward_noalloc: batch < 1 or NULL argument");
    if (n_sym < 1 || n_sym > 8) return set_error(LBM_EINVAL, "lbm_cnn_forward_noalloc: n_sym must lie in [1, 8]");
    if (max_workgroups < 0) return set_error(LBM_EINVAL, "lbm_cnn_forward_noalloc: max_workgroups must be >= 0");
    const SurLayout L = sur_layout(batch, false);
    if (L.total > kNoAllocScratchBytes)
        return set_error(LBM_EINVAL, "lbm_cnn_forward_noalloc: the call needs " + std::to_string(L.total) +
                                         " bytes of scratch, more than the " +
                                         std::to_string(kNoAllocScratchBytes) + " reserved");
    void *p = nullptr;
    lbm_status s = scratch_address(&p);
    if (s != LBM_OK) return s;
    char *ws = static_cast<char *>(p);
    s = pack(d_params, ws, L, stream);  // also zeroes the patch counter
    if (s != LBM_OK) return s;
    return forward(d_params, batch, d_logk, nullptr, n_sym, d_pred, d_stats, ws, L, false, stream,
                   max_workgroups);
}

extern "C" lbm_status lbm_cnn_forward_spread(const float *d_params, int32_t batch, const float *d_logk,
                                             int32_t n_sym, float *d_pred, float *d_spread, int32_t max_workgroups,
                                             void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    if (batch < 1 || !d_params || !d_logk || !d_pred || !d_spread)
        return set_error(LBM_EINVAL, "lbm_cnn_forward_spread: batch < 1 or NULL argument");
    if (n_sym < 1 || n_sym > 8) return set_error(LBM_EINVAL, "lbm_cnn_forward_spread: n_sym must lie in [1, 8]");
    if (max_workgroups < 0) return set_error(LBM_EINVAL, "lbm_cnn_forward_spread: max_workgroups must be >= 0");
    const SurLayout L = sur_layout(batch, false);
    lbm_status s = check_ws(d_ws, ws_bytes, L.total, "lbm_cnn_forward_spread");
    if (s != LBM_OK) return s;
    char *ws = static_cast<char *>(d_ws);
    s = pack(d_params, ws, L, stream);
    if (s != LBM_OK) return s;
    return forward(d_params, batch, d_logk, nullptr, n_sym, d_pred, nullptr, ws, L, false, stream, max_workgroups,
                   d_spread);
}

extern "C" lbm_status lbm_cnn_forward(const float *d_params, int32_t batch, const float *d_logk, int32_t n_sym,
                                      float *d_pred, float *d_stats, void *d_ws, size_t ws_bytes,
                                      hipStream_t stream)
{
    return lbm_cnn_forward_limited(d_params, batch, d_logk, n_sym, d_pred, d_stats, 0, d_ws, ws_bytes, stream);
}

extern "C" lbm_status lbm_cnn_gradients(const float *d_params, int32_t batch, const float *d_logk,
                                        const int8_t *d_sym, const float *d_target, float *d_grad, float *d_loss,
                                        float *d_pred, void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    if (batch < 1 || !d_params || !d_logk || !d_target || !d_pred)
        return set_error(LBM_EINVAL, "lbm_cnn_gradients: batch < 1 or NULL argument");
    const SurLayout L = sur_layout(batch, true);
    lbm_status s = check_ws(d_ws, ws_bytes, L.total, "lbm_cnn_gradients");
    if (s != LBM_OK) return s;
    char *ws = static_cast<char *>(d_ws);
    s = gradients(d_params, batch, d_logk, d_sym, d_target, d_pred, ws, L, stream);
    if (s != LBM_OK) return s;
    if (d_grad)
        LBM_HIP(hipMemcpyAsync(d_grad, ws + L.off_grad, kNParams * 4, hipMemcpyDeviceToDevice, stream));
    if (d_loss) LBM_HIP(hipMemcpyAsync(d_loss, ws + L.off_loss, 4, hipMemcpyDeviceToDevice, stream));
    return LBM_OK;
}

extern "C" lbm_status lbm_cnn_train_step(float *d_params, float *d_adam_m, float *d_adam_v, int32_t step, float lr,
                                         int32_t batch, const float *d_logk, const int8_t *d_sym,
                                         const float *d_target, float *d_loss, void *d_ws, size_t ws_bytes,
                                         hipStream_t stream)
{
    if (batch < 1 || !d_params || !d_adam_m || !d_adam_v || !d_logk || !d_target || step < 1 || !(lr > 0.0f))
        return set_error(LBM_EINVAL, "lbm_cnn_train_step: bad argument");
    const SurLayout L = sur_layout(batch, true);
    lbm_status s = check_ws(d_ws, ws_bytes, L.total, "lbm_cnn_train_step");
    if (s != LBM_OK) return s;
    char *ws = static_cast<char *>(d_ws);
    float *pred = reinterpret_cast<float *>(ws + L.off_pred);
    s = gradients(d_params, batch, d_logk, d_sym, d_target, pred, ws, L, stream);
    if (s != LBM_OK) return s;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((kNParams + 255) / 256), dim3(256), 0, stream, d_params, d_adam_m, d_adam_v,
                       reinterpret_cast<const float *>(ws + L.off_grad), lr, b1, b2, 1e-8f, c1, c2);
    LBM_HIP(hipGetLastError());
    if (d_loss) LBM_HIP(hipMemcpyAsync(d_loss, ws + L.off_loss, 4, hipMemcpyDeviceToDevice, stream));
    return LBM_OK;
}
