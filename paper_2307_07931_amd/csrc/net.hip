// net.hip -- the learned correction network: forward, backward and Adam on gfx950.
//
// Network (not from the paper; an extension): x -> conv3x3 1->32 -> ReLU ->
// conv3x3 32->32 -> ReLU -> conv3x3 32->32 -> ReLU -> conv3x3 32->1 -> y, no bias,
// zero padding.  BF16 weights and activations, FP32 accumulation.
//
// * The two 32->32 layers (96% of the arithmetic) run as implicit GEMMs on the
//   matrix cores: one wavefront computes 32 output channels x 32 pixels of one
//   image row with v_mfma_f32_32x32x16_bf16, K = 9 taps x 32 channels = 18
//   instructions.  The same kernel computes the input gradient (transposed
//   convolution: taps mirrored, weights in [tap][in][out] order) with the ReLU
//   mask of the layer's input applied in the epilogue.
// * Layer 1 (1 input channel) and layer 4 (1 output channel) are thin; they run on
//   the vector ALUs.
// * Weight gradients are reductions over all pixels: every block sums a fixed
//   pixel range into private partials, and a second kernel adds the partials in
//   block order, so results are deterministic.
// Activations are stored channels-last (pixel-major, 32 channels = 64 bytes).
#include "../../include/protox.h"
#include "px_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace px {
namespace {

constexpr int C = 32;          // hidden channels
constexpr int NW1 = C * 9;     // layer 1 weights
constexpr int NW2 = C * C * 9; // layer 2 / 3 weights
constexpr int NW4 = C * 9;     // layer 4 weights
constexpr int NPARAM = NW1 + 2 * NW2 + NW4;  // 19008
constexpr int OFF2 = NW1, OFF3 = NW1 + NW2, OFF4 = NW1 + 2 * NW2;
constexpr int WT_ROWS = 4;      // image rows per work unit of the thin layers' weight gradients
constexpr int WT_WAVES = 8192;  // at most this many waves (and partial slots) for them
constexpr int RS = 32;          // first-pass slices of the partial-sum reduction (32 -> 32 layers)
constexpr int RS_THIN = 64;     // the same for the thin layers' 288 sums
static_assert(RS_THIN * NW1 <= RS * NW2, "both slicings fit the middle buffer");
constexpr int BX = 256;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bfv(bf16 x) { return bf16_to_f32(x.bits); }
__device__ __forceinline__ bf16 tobf(float x) { return bf16{f32_to_bf16_rne(x)}; }
// ReLU that keeps NaN (as max(x, 0) of IEEE propagation would): a broken network stays visible.
__device__ __forceinline__ float relu(float x) { return x < 0.0f ? 0.0f : x; }

// tap t = 3a + c reads offset (a - 1, c - 1); the transposed convolution reads (1 - a, 1 - c)
__device__ __forceinline__ int tap_dy(int t, bool mirror) { return mirror ? 1 - t / 3 : t / 3 - 1; }
__device__ __forceinline__ int tap_dx(int t, bool mirror) { return mirror ? 1 - t % 3 : t % 3 - 1; }

struct NetW {
    bf16 *w1;   // [co][t]
    bf16 *w2f;  // [t][co][ci]  (forward: rows = output channel, k = input channel)
    bf16 *w2b;  // [t][ci][co]  (input gradient: rows = input channel, k = output channel)
    bf16 *w3f, *w3b;
    bf16 *w4;   // [ci][t]
};

__global__ __launch_bounds__(BX) void prep_weights_kernel(const float *__restrict__ w, NetW nw)
{
    const int q = blockIdx.x * BX + threadIdx.x;
    if (q >= NPARAM) return;
    const bf16 b = tobf(w[q]);
    if (q < OFF2) {
        nw.w1[q] = b;  // (co, 1, a, c) -> co*9 + t
    } else if (q < OFF4) {
        const bool l3 = q >= OFF3;
        const int r = q - (l3 ? OFF3 : OFF2);
        const int co = r / (C * 9), ci = (r / 9) % C, t = r % 9;
        (l3 ? nw.w3f : nw.w2f)[(t * C + co) * C + ci] = b;
        (l3 ? nw.w3b : nw.w2b)[(t * C + ci) * C + co] = b;
    } else {
        nw.w4[q - OFF4] = b;  // (1, ci, a, c) -> ci*9 + t
    }
}

// Tiles of the thin layers: a block of BX threads owns 4 rows x 64 pixels, one pixel per
// thread; the input patch (1-pixel halo) and the layer's weights are staged in LDS.
constexpr int LT_ROWS = 4, LT_PX = 64;
static_assert(LT_ROWS * LT_PX == BX, "one pixel per thread");

// Layer 1 on the matrix cores, 32 pixels per v_mfma_f32_32x32x16_bf16: rows = the 32
// output channels, columns = the pixels, k = the 9 taps (then 7 zeros).  l1_weights gives
// a lane's part of the weight operand (row lane mod 32, taps 8 (lane / 32) + 0..7);
// l1_group takes the lane's eight inputs of its pixel (column lane mod 32) at those taps
// and returns the products (the lane's channels 8g + 4 (lane / 32) + e in element 4g + e).
// The layer-1 kernel and the fused first convolution both use them, so both produce the
// same bits.
__device__ __forceinline__ bf16x8 l1_weights(const bf16 *__restrict__ w1)
{
    const int lane = threadIdx.x & 63, co = lane & 31, kg = lane >> 5;
    bf16x8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int t = 8 * kg + e;
        a[e] = __builtin_bit_cast(__bf16, t < 9 ? w1[co * 9 + t].bits : (uint16_t)0);
    }
    return a;
}

__device__ __forceinline__ f32x16 l1_group(const bf16x8 &aw, const float (&xt)[8])
{
    bf16x8 b;
#pragma unroll
    for (int e = 0; e < 8; ++e) b[e] = __builtin_bit_cast(__bf16, (uint16_t)(__float_as_uint(xt[e]) >> 16));
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw, b, f32x16{}, 0, 0, 0);
}

// The lane's 16 channels of its pixel after ReLU, rounded to BF16, at dst (a pixel's
// channel row), as four 8-byte stores.
__device__ __forceinline__ void l1_store(const f32x16 &acc, bool zero, bf16 *dst)
{
    const int kg = (threadIdx.x & 63) >> 5;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        unsigned short v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = zero ? (unsigned short)0 : f32_to_bf16_rne(relu(acc[4 * g + e]));
        uint2 pk;
        pk.x = (unsigned)v[0] | ((unsigned)v[1] << 16);
        pk.y = (unsigned)v[2] | ((unsigned)v[3] << 16);
        *reinterpret_cast<uint2 *>(dst + 8 * g + 4 * kg) = pk;
    }
}

// The first layer's input: x (FP64 or FP32) times `scale`, rounded to FP32, then to BF16.
template <typename TX> __device__ __forceinline__ float l1_input(TX v, double scale)
{
    return bf16_to_f32(f32_to_bf16_rne((float)((double)v * scale)));
}

// Layer 1: x (rows of ldx, FP64 or FP32) times `scale`, rounded to FP32 and then to
// BF16, -> 32 channels, ReLU, on the matrix cores (l1_group).  One block per tile of
// 4 rows x 64 pixels: the input patch (1-pixel halo) is staged in LDS, each wave forms two
// 32-pixel groups, and the results go through LDS so that every store instruction of a
// wave writes 1 KB of consecutive memory (16 pixels of one row).
template <typename TX>
__global__ __launch_bounds__(BX) void l1_fwd_kernel(const TX *__restrict__ x, int ldx, double scale,
                                                    const bf16 *__restrict__ w1, bf16 *__restrict__ a1, int B,
                                                    int H, int W)
{
    constexpr int SXC = LT_PX + 2;
    constexpr int OSTR = 40;  // pixel slots of the output staging, padded to 80 bytes
    __shared__ float sx[(LT_ROWS + 2) * SXC];
    __shared__ __align__(16) bf16 so[LT_ROWS * LT_PX * OSTR];
    const int tiles_w = (W + LT_PX - 1) / LT_PX, tiles_h = (H + LT_ROWS - 1) / LT_ROWS;
    const int tw = (int)(blockIdx.x % tiles_w), th = (int)((blockIdx.x / tiles_w) % tiles_h);
    const int b = (int)(blockIdx.x / ((unsigned)tiles_w * tiles_h));
    const int i0 = th * LT_ROWS, j0 = tw * LT_PX;
    const bf16x8 aw = l1_weights(w1);
    for (int q = threadIdx.x; q < (LT_ROWS + 2) * SXC; q += BX) {
        const int pr = q / SXC, pc = q % SXC;
        const int ii = i0 - 1 + pr, jj = j0 - 1 + pc;
        float v = 0.0f;
        if (ii >= 0 && ii < H && jj >= 0 && jj < W) v = l1_input(x[((long long)b * H + ii) * ldx + jj], scale);
        sx[q] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, kg = lane >> 5;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int px = (2 * wv + h) * 32 + (lane & 31);  // pixel of the tile, row-major
        const int r = px / LT_PX, c = px % LT_PX;
        float xt[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int t = 8 * kg + e;
            xt[e] = t < 9 ? sx[(r + 1 + tap_dy(t, false)) * SXC + (c + 1 + tap_dx(t, false))] : 0.0f;
        }
        l1_store(l1_group(aw, xt), false, so + px * OSTR);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int chunk = q * BX + (int)threadIdx.x;  // 16-byte piece of the tile, row-major
        const int row = chunk / (LT_PX * 4), px = (chunk / 4) % LT_PX, part = chunk % 4;
        const int ii = i0 + row, jj = j0 + px;
        if (ii < H && jj < W)
            *reinterpret_cast<uint4 *>(a1 + (((long long)b * H + ii) * W + jj) * C + part * 8) =
                *reinterpret_cast<const uint4 *>(so + (row * LT_PX + px) * OSTR + part * 8);
    }
}

// 32 -> 32 convolution on the matrix cores, as an implicit GEMM per output tile.
//
// A block (4 waves) owns TROWS = 4 image rows x TPX = 64 pixels; wave w computes row
// i0 + w, as two 32-pixel halves.  The block stages the input patch it needs
// ((TROWS + 2) x (TPX + 2) pixels x 32 channels) and the layer's weights (9 taps x 32 x
// 32) in LDS once, then each wave runs 9 taps x 2 channel halves x 2 pixel halves = 36
// v_mfma_f32_32x32x16_bf16: A = weights (rows: output channel, k: input channel of the
// tap), B = patch pixels (k: input channel, columns: pixel), operands read from LDS with
// 16-byte loads.  Pixels and weight rows are padded to PSTR = 40 elements (80 bytes) so
// that the 16-byte reads of neighbouring lanes fall in different LDS banks.  Blocks
// loop over tiles so the weights are loaded once per block.
//
// MIRROR computes the input gradient: `in` is the gradient of the layer output, the
// weights are in [t][ci][co] order, the taps are mirrored, and the result is multiplied
// by the ReLU mask of `mask` (the layer's input activation).  Otherwise the epilogue
// applies ReLU.  Outputs are rounded to BF16 and stored channels-last.
constexpr int TROWS = 4, TPX = 64, PSTR = 40;
constexpr int PROWS = TROWS + 2, PCOLS = TPX + 2;

constexpr int PCHUNKS = PROWS * PCOLS * 4;            // 16-byte chunks of one patch
constexpr int PPER = (PCHUNKS + BX - 1) / BX;         // chunks per thread

// Issue the global loads of one tile's patch into registers (zeros outside the image).
__device__ __forceinline__ void patch_load(const bf16 *__restrict__ in, int tile, int tiles_w, int tiles_h, int H,
                                           int W, uint4 (&reg)[PPER])
{
    const int tw = tile % tiles_w, th = (tile / tiles_w) % tiles_h, b = tile / (tiles_w * tiles_h);
    const int i0 = th * TROWS, j0 = tw * TPX;
#pragma unroll
    for (int u = 0; u < PPER; ++u) {
        const int q = (int)threadIdx.x + u * BX;
        reg[u] = make_uint4(0, 0, 0, 0);
        if (q < PCHUNKS) {
            const int ch = q & 3, pc = (q >> 2) % PCOLS, pr = (q >> 2) / PCOLS;
            const int ii = i0 - 1 + pr, jj = j0 - 1 + pc;
            if (ii >= 0 && ii < H && jj >= 0 && jj < W)
                reg[u] = *reinterpret_cast<const uint4 *>(in + (((long long)b * H + ii) * W + jj) * C + ch * 8);
        }
    }
}

// Orders a wave's LDS writes before its later LDS reads of other lanes' data (the LDS
// serves one wave's instructions in order; this only stops the compiler moving them).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The matrix products and the epilogue of one tile, its patch and the weights in LDS.
// The epilogue goes through `so` (TROWS x TPX pixels, PSTR elements each; wave w uses
// row w only): each lane leaves its results there and the wave then writes its row with
// 16-byte stores of consecutive memory (1 KB per store instruction), where storing from
// the accumulators directly scatters 8 bytes per lane over 32 pixels.  The backward's
// ReLU mask comes in the same way, with coalesced loads.
// A wave's weight operands for all 9 taps x 2 channel halves (72 registers), read from the
// staged weights once per block and kept for every tile the block computes.
struct ConvA {
    bf16x8 a[9][2];
};
__device__ __forceinline__ void load_conv_weights(const bf16 *__restrict__ sw, ConvA &w)
{
    const int lane = threadIdx.x & 63, n = lane & 31, kg = lane >> 5;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int c16 = 0; c16 < 2; ++c16) __builtin_memcpy(&w.a[t][c16], sw + (t * C + n) * PSTR + c16 * 16 + kg * 8, 16);
}

template <bool MIRROR>
__device__ __forceinline__ void conv32_tile(const ConvA &w, const bf16 *__restrict__ sp, bf16 *__restrict__ so,
                                            int tile, int tiles_w, int tiles_h, int H, int W, bf16 *__restrict__ out,
                                            const bf16 *__restrict__ mask)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = lane & 31, kg = lane >> 5;
    const int tw = tile % tiles_w, th = (tile / tiles_w) % tiles_h, b = tile / (tiles_w * tiles_h);
    const int i0 = th * TROWS, j0 = tw * TPX;
    f32x16 acc0 = {}, acc1 = {};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int pr = wv + 1 + tap_dy(t, MIRROR), pc = n + 1 + tap_dx(t, MIRROR);
#pragma unroll
        for (int c16 = 0; c16 < 2; ++c16) {
            const int k0 = c16 * 16 + kg * 8;
            bf16x8 b0, b1;
            __builtin_memcpy(&b0, sp + (pr * PCOLS + pc) * PSTR + k0, 16);
            __builtin_memcpy(&b1, sp + (pr * PCOLS + pc + 32) * PSTR + k0, 16);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w.a[t][c16], b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w.a[t][c16], b1, acc1, 0, 0, 0);
        }
    }
    const int i = i0 + wv;
    if (i >= H) return;
    bf16 *row = so + wv * TPX * PSTR;
    const long long p0 = ((long long)b * H + i) * W + j0;  // the row's first pixel
    const int nvalid = min(TPX, W - j0);
    if (MIRROR) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int chunk = q * 64 + lane, px = chunk >> 2, part = chunk & 3;
            if (px < nvalid)
                *reinterpret_cast<uint4 *>(row + px * PSTR + part * 8) =
                    *reinterpret_cast<const uint4 *>(mask + (p0 + px) * C + part * 8);
        }
        wave_lds_sync();
    }
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const f32x16 &acc = half ? acc1 : acc0;
        // lane holds output channels 8g + 4 kg + e (e = 0..3) of pixel half*32 + n in acc[4g + e]
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int co = 8 * g + 4 * kg;
            uint2 *slot = reinterpret_cast<uint2 *>(row + (half * 32 + n) * PSTR + co);
            uint2 mk = make_uint2(0, 0);
            if (MIRROR) mk = *slot;  // this lane's own four mask values, overwritten below
            unsigned short v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float a = acc[4 * g + e];
                if (MIRROR) {
                    const unsigned mb = ((e < 2 ? mk.x : mk.y) >> (16 * (e & 1))) & 0xffffu;
                    a = bf16_to_f32((unsigned short)mb) > 0.0f ? a : 0.0f;
                } else {
                    a = relu(a);
                }
                v[e] = f32_to_bf16_rne(a);
            }
            uint2 pk;
            pk.x = (unsigned)v[0] | ((unsigned)v[1] << 16);
            pk.y = (unsigned)v[2] | ((unsigned)v[3] << 16);
            *slot = pk;
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int chunk = q * 64 + lane, px = chunk >> 2, part = chunk & 3;
        if (px < nvalid)
            *reinterpret_cast<uint4 *>(out + (p0 + px) * C + part * 8) =
                *reinterpret_cast<const uint4 *>(row + px * PSTR + part * 8);
    }
}

// The layer's weights into LDS, rows padded to PSTR elements.
__device__ __forceinline__ void stage_weights(const bf16 *__restrict__ wl, bf16 *__restrict__ sw)
{
    for (int q = threadIdx.x; q < 9 * C * 4; q += BX) {
        const int row = q >> 2, ch = q & 3;
        *reinterpret_cast<uint4 *>(sw + row * PSTR + ch * 8) = *reinterpret_cast<const uint4 *>(wl + row * C + ch * 8);
    }
}

template <bool MIRROR>
__global__ __launch_bounds__(BX) void conv32_kernel(const bf16 *__restrict__ in, const bf16 *__restrict__ wl,
                                                    bf16 *__restrict__ out, const bf16 *__restrict__ mask, int B,
                                                    int H, int W)
{
    __shared__ __align__(16) bf16 sw[9 * C * PSTR];
    __shared__ __align__(16) bf16 sp[PROWS * PCOLS * PSTR];
    __shared__ __align__(16) bf16 so[TROWS * TPX * PSTR];
    const int tid = threadIdx.x;
    stage_weights(wl, sw);
    __syncthreads();
    ConvA wr;
    load_conv_weights(sw, wr);
    const int tiles_w = (W + TPX - 1) / TPX, tiles_h = (H + TROWS - 1) / TROWS;
    const int ntiles = B * tiles_h * tiles_w;  // < 2^31: at most 2^31 pixels
    uint4 reg[PPER];
    if ((int)blockIdx.x < ntiles) patch_load(in, blockIdx.x, tiles_w, tiles_h, H, W, reg);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        __syncthreads();  // the previous tile's LDS reads are done (first pass: weights stored)
#pragma unroll
        for (int u = 0; u < PPER; ++u) {
            const int q = tid + u * BX;
            if (q < PCHUNKS) {
                const int ch = q & 3, pix = q >> 2;
                *reinterpret_cast<uint4 *>(sp + pix * PSTR + ch * 8) = reg[u];
            }
        }
        __syncthreads();
        // the next tile's patch loads fly while this tile's matrix products run
        if (tile + (int)gridDim.x < ntiles) patch_load(in, tile + gridDim.x, tiles_w, tiles_h, H, W, reg);
        conv32_tile<MIRROR>(wr, sp, so, tile, tiles_w, tiles_h, H, W, out, mask);
    }
}

// Layers 1 and 2 in one pass (inference: the layer-1 activations are not kept).  Per tile
// the block stages the input x of the patch's neighbourhood ((PROWS + 2) x (PCOLS + 2)
// pixels, rounded as the first layer's input), computes layer 1 for the PROWS x PCOLS
// patch pixels with l1_group straight into the patch buffer (zero outside the image, the
// second layer's zero padding), then runs the second layer's matrix products as
// conv32_kernel does.  The patch holds exactly the values l1_fwd_kernel would have
// stored, so the output equals l1_fwd_kernel followed by conv32_kernel bit for bit, with
// the 64-byte-per-pixel layer-1 activations never written to or read from memory.
constexpr int XROWS = PROWS + 2, XCOLS = PCOLS + 2;
constexpr int L1_GROUPS = (PROWS * PCOLS + 31) / 32;  // 32-pixel groups of layer 1 per patch
template <typename TX>
__global__ __launch_bounds__(BX) void conv12_kernel(const TX *__restrict__ x, int ldx, double scale,
                                                    const bf16 *__restrict__ w1, const bf16 *__restrict__ wl,
                                                    bf16 *__restrict__ out, int B, int H, int W)
{
    __shared__ __align__(16) bf16 sw[9 * C * PSTR];
    __shared__ __align__(16) bf16 sp[PROWS * PCOLS * PSTR];
    __shared__ float sx[XROWS * XCOLS];
    __shared__ __align__(16) bf16 so[TROWS * TPX * PSTR];
    const int tid = threadIdx.x;
    stage_weights(wl, sw);
    __syncthreads();
    ConvA wr;
    load_conv_weights(sw, wr);
    const bf16x8 aw = l1_weights(w1);
    const int tiles_w = (W + TPX - 1) / TPX, tiles_h = (H + TROWS - 1) / TROWS;
    const int ntiles = B * tiles_h * tiles_w;
    // x of a tile's neighbourhood, XPER values per thread, loaded one tile ahead (in flight
    // during the current tile's layer 1 and matrix products); `inside` says which of them
    // lie in the image (the others stand for the zero padding)
    constexpr int XPER = (XROWS * XCOLS + BX - 1) / BX;
    TX xr[XPER];
    bool inside[XPER];
    auto xload = [&](int t) {
        const int tw = t % tiles_w, th = (t / tiles_w) % tiles_h, b = t / (tiles_w * tiles_h);
        const int i0 = th * TROWS, j0 = tw * TPX;
#pragma unroll
        for (int u = 0; u < XPER; ++u) {
            const int q = tid + u * BX;
            const int ii = i0 - 2 + q / XCOLS, jj = j0 - 2 + q % XCOLS;
            inside[u] = q < XROWS * XCOLS && ii >= 0 && ii < H && jj >= 0 && jj < W;
            xr[u] = inside[u] ? x[((long long)b * H + ii) * ldx + jj] : (TX)0;
        }
    };
    if ((int)blockIdx.x < ntiles) xload(blockIdx.x);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tw = tile % tiles_w, th = (tile / tiles_w) % tiles_h;
        const int i0 = th * TROWS, j0 = tw * TPX;
        __syncthreads();  // the previous tile's reads of sx and sp are done
#pragma unroll
        for (int u = 0; u < XPER; ++u) {
            const int q = tid + u * BX;
            if (q < XROWS * XCOLS) sx[q] = inside[u] ? l1_input(xr[u], scale) : 0.0f;
        }
        __syncthreads();
        if (tile + (int)gridDim.x < ntiles) xload(tile + gridDim.x);
        // layer 1 for the patch pixels, 32 per group; pixels outside the image are the
        // second layer's zero padding
        for (int g = tid >> 6; g < L1_GROUPS; g += BX / 64) {
            const int px = g * 32 + (tid & 31);
            const bool valid = px < PROWS * PCOLS;
            const int pxc = valid ? px : 0;  // columns past the patch compute pixel 0, unused
            const int pr = pxc / PCOLS, pc = pxc % PCOLS;
            const int ii = i0 - 1 + pr, jj = j0 - 1 + pc;
            float xt[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int t = 8 * ((tid & 63) >> 5) + e;
                xt[e] = t < 9 ? sx[(pr + 1 + tap_dy(t, false)) * XCOLS + (pc + 1 + tap_dx(t, false))] : 0.0f;
            }
            const f32x16 acc = l1_group(aw, xt);
            if (valid) l1_store(acc, !(ii >= 0 && ii < H && jj >= 0 && jj < W), sp + px * PSTR);
        }
        __syncthreads();
        conv32_tile<false>(wr, sp, so, tile, tiles_w, tiles_h, H, W, out, nullptr);
    }
}

// Layer 4: 32 channels -> 1, output FP32 into rows of ldy, on the matrix cores.  With
// z_t(q) = sum over the 32 input channels of w4[ci][t] a3(q, ci), the output is
// y(p) = z_0(p + o_0) + ... + z_8(p + o_8) (o_t the tap offsets, taps in order).  Tiles of
// 4 rows x 64 pixels (the convolution's): the block stages the a3 patch (6 x 66 pixels,
// rows padded to PSTR elements), forms z for all nine taps at every patch pixel as
// v_mfma_f32_16x16x32_bf16 products (rows: taps, 9 of 16 used; columns: 16 patch pixels;
// k: the 32 channels) into LDS, and each thread then adds its pixel's nine z values.
// Blocks loop over tiles with the next tile's patch loads in flight, as the convolution
// does.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int L4_NPIX = PROWS * PCOLS;         // patch pixels
constexpr int L4_GROUPS = (L4_NPIX + 15) / 16;  // 16-pixel column groups of the products
// row pitch of the per-tap sums in LDS: 4 mod 16 words, so the four taps a product writes
// at once (rows 4 kq + e, 16 pixels each) start in different banks
constexpr int L4_ZSTR = L4_GROUPS * 16 + 4;
__global__ __launch_bounds__(BX) void l4_fwd_kernel(const bf16 *__restrict__ a3, const bf16 *__restrict__ w4,
                                                    float *__restrict__ y, int ldy, int B, int H, int W)
{
    static_assert(LT_ROWS == TROWS && LT_PX == TPX, "layer 4 uses the convolution's tiles and patches");
    __shared__ __align__(16) bf16 sp[L4_NPIX * PSTR];
    __shared__ float sz[9][L4_ZSTR];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;  // product column (pixel of the group); k and row quarter
    // A: row = tap col (taps 9..15 zero), k = channels 8 kq .. 8 kq + 7
    bf16x8 aw;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const bf16 wt = col < 9 ? w4[(8 * kq + e) * 9 + col] : bf16{0};
        aw[e] = __builtin_bit_cast(__bf16, wt.bits);
    }
    const int tiles_w = (W + TPX - 1) / TPX, tiles_h = (H + TROWS - 1) / TROWS;
    const int ntiles = B * tiles_h * tiles_w;
    const int r = threadIdx.x / TPX, c = threadIdx.x % TPX;
    uint4 reg[PPER];
    if ((int)blockIdx.x < ntiles) patch_load(a3, blockIdx.x, tiles_w, tiles_h, H, W, reg);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tw = tile % tiles_w, th = (tile / tiles_w) % tiles_h, b = tile / (tiles_w * tiles_h);
        __syncthreads();  // the previous tile's reads of sp and sz are done
#pragma unroll
        for (int u = 0; u < PPER; ++u) {
            const int q = (int)threadIdx.x + u * BX;
            if (q < PCHUNKS) {
                const int ch = q & 3, pix = q >> 2;
                *reinterpret_cast<uint4 *>(sp + pix * PSTR + ch * 8) = reg[u];
            }
        }
        __syncthreads();
        if (tile + (int)gridDim.x < ntiles) patch_load(a3, tile + gridDim.x, tiles_w, tiles_h, H, W, reg);
        for (int g = wv; g < L4_GROUPS; g += BX / 64) {
            const int px = g * 16 + col;
            const int pxr = px < L4_NPIX ? px : 0;  // columns past the patch read pixel 0, unused
            bf16x8 bv;
            __builtin_memcpy(&bv, sp + pxr * PSTR + 8 * kq, 16);
            const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bv, f32x4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
            // lane holds rows (taps) 4 kq + e of column col
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (4 * kq + e < 9) sz[4 * kq + e][px] = d[e];
        }
        __syncthreads();
        const int i = th * TROWS + r, j = tw * TPX + c;
        if (i >= H || j >= W) continue;
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc += sz[t][(r + 1 + tap_dy(t, false)) * PCOLS + (c + 1 + tap_dx(t, false))];
        y[((long long)b * H + i) * ldy + j] = acc;
    }
}

// Fixed-order block reduction of one double per thread; thread 0 gets the total.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = BX / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + h];
        __syncthreads();
    }
    return sh[0];
}

// Mean squared error: dy = 2 (y - t) / N, per-block partial sums of (y - t)^2.
__global__ __launch_bounds__(BX) void mse_kernel(const float *__restrict__ y, const float *__restrict__ tg,
                                                 float *__restrict__ dy, double *__restrict__ part, long long N)
{
    __shared__ double sh[BX];
    const long long p = (long long)blockIdx.x * BX + threadIdx.x;
    double e2 = 0.0;
    if (p < N) {
        const float d = y[p] - tg[p];
        dy[p] = (float)(2.0 / (double)N) * d;
        e2 = (double)d * (double)d;
    }
    const double tot = block_sum(e2, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Energy loss, first pass: y <- y - t.
__global__ __launch_bounds__(BX) void diff_kernel(float *__restrict__ y, const float *__restrict__ tg, long long N)
{
    const long long p = (long long)blockIdx.x * BX + threadIdx.x;
    if (p < N) y[p] = y[p] - tg[p];
}

// Energy loss, second pass on d = y - t: kd = 4 d - (sum of the 4 neighbours), a
// neighbour outside the image being -d (odd reflection); dy = 2 kd / N, partial sums of
// d * kd.
__global__ __launch_bounds__(BX) void energy_kernel(const float *__restrict__ d, float *__restrict__ dy,
                                                    double *__restrict__ part, int B, int H, int W)
{
    __shared__ double sh[BX];
    const long long N = (long long)B * H * W;
    const long long p = (long long)blockIdx.x * BX + threadIdx.x;
    double e = 0.0;
    if (p < N) {
        const int j = (int)(p % W), i = (int)((p / W) % H);
        const float c = d[p];
        const float dn = i > 0 ? d[p - W] : -c;
        const float ds = i < H - 1 ? d[p + W] : -c;
        const float dw = j > 0 ? d[p - 1] : -c;
        const float de = j < W - 1 ? d[p + 1] : -c;
        const float kd = 4.0f * c - (((dn + dw) + de) + ds);
        dy[p] = (float)(2.0 / (double)N) * kd;
        e = (double)c * (double)kd;
    }
    const double tot = block_sum(e, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(BX) void sum_partials_kernel(const double *__restrict__ part, int count,
                                                          double *__restrict__ out, double mul)
{
    __shared__ double sh[BX];
    double s = 0.0;
    for (int k = threadIdx.x; k < count; k += BX) s = s + part[k];
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) *out = tot * mul;
}

// Two fixed-order sums of double2 partials: out[0] = sum .x, out[1] = sum .y.
__global__ __launch_bounds__(BX) void sum2_partials_kernel(const double2 *__restrict__ part, int count,
                                                           double *__restrict__ out)
{
    __shared__ double sh[BX];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < count; k += BX) {
        a = a + part[k].x;
        b = b + part[k].y;
    }
    const double ta = block_sum(a, sh);
    __syncthreads();
    const double tb = block_sum(b, sh);
    if (threadIdx.x == 0) {
        out[0] = ta;
        out[1] = tb;
    }
}

// Layer-4 input gradient: dz3[p][ci] = (sum_t dy[p - off_t] w4[ci][t]) * (a3[p][ci] > 0).
__global__ __launch_bounds__(BX) void l4_bwd_kernel(const float *__restrict__ dy, const bf16 *__restrict__ w4,
                                                    const bf16 *__restrict__ a3, bf16 *__restrict__ dz3, int B,
                                                    int H, int W)
{
    const long long p = (long long)blockIdx.x * BX + threadIdx.x;
    if (p >= (long long)B * H * W) return;
    const int j = (int)(p % W), i = (int)((p / W) % H), b = (int)(p / ((long long)W * H));
    float d[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int ii = i + tap_dy(t, true), jj = j + tap_dx(t, true);
        d[t] = (ii >= 0 && ii < H && jj >= 0 && jj < W) ? dy[((long long)b * H + ii) * W + jj] : 0.0f;
    }
    bf16 out[C];
#pragma unroll
    for (int ci = 0; ci < C; ++ci) {
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc += d[t] * bfv(w4[ci * 9 + t]);
        out[ci] = tobf(bfv(a3[p * C + ci]) > 0.0f ? acc : 0.0f);
    }
    uint4 *dst = reinterpret_cast<uint4 *>(dz3 + p * C);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = reinterpret_cast<const uint4 *>(out)[q];
}

// Weight gradient of a 32 -> 32 layer on the matrix cores:
//   dW[co][ci][t] = sum_p dz[p][co] act[p + (a - 1, c - 1)][ci],   t = 3a + c.
// With q = p + (0, c - 1) the sum runs over q with dz[q - (0, c - 1)] and act[q + (a - 1, 0)]:
// the column shift moves to dz, so the activation operand is read at aligned pixels (terms
// with q outside [0, W) meet the zero padding of act).  Per tap it is a 32 x 32 GEMM over
// pixels, K = pixels, which the matrix cores read 8 consecutive K values per lane: the wave
// stages its operands in LDS channel-major.  A wave (one per block) owns a 64-pixel column
// strip of WG_ROWS image rows; per row i it stages activation row i + 1 (rows i - 1, i, i + 1
// form a ring) and dz row i in three copies shifted by c - 1, then runs 9 taps x 4 chunks of
// 16 pixels = 36 v_mfma_f32_32x32x16_bf16 into 9 accumulator tiles.  Blocks take work units
// in a fixed order and write one partial each; a second pass sums them in block order.
constexpr int WGP = 72;        // pixels per channel row in LDS (64 + pad: conflict-free reads)
constexpr int WG_ROWS = 16;    // image rows per work unit
constexpr int WGM_BLOCKS = 2048;

__global__ __launch_bounds__(64) void wgrad32_mfma_kernel(const bf16 *__restrict__ act,
                                                          const bf16 *__restrict__ dz, float *__restrict__ part,
                                                          int B, int H, int W)
{
    __shared__ __align__(16) bf16 sa[3][C][WGP];  // activation rows, slot = row mod 3
    __shared__ __align__(16) bf16 sd[3][C][WGP];  // sd[c][co][px] = dz[i][j0 + px - (c - 1)][co]
    const int lane = threadIdx.x;
    const int n = lane & 31, kg = lane >> 5;
    const int strips = (W + 63) / 64, groups = (H + WG_ROWS - 1) / WG_ROWS;
    const int units = B * strips * groups;
    f32x16 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x16{};

    // one pixel's 32 channels of row ii of image b (zeros outside the image) into LDS
    // column pos of the channel-major rows at dst (row stride WGP)
    auto put = [&](bf16 *dst, const bf16 *src, int b, int ii, int jj, int pos) {
        uint4 v[4] = {make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0)};
        if (ii >= 0 && ii < H && jj >= 0 && jj < W) {
            const uint4 *g = reinterpret_cast<const uint4 *>(src + (((long long)b * H + ii) * W + jj) * C);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = g[q];
        }
        const unsigned short *h = reinterpret_cast<const unsigned short *>(v);
#pragma unroll
        for (int ch = 0; ch < C; ++ch) dst[ch * WGP + pos] = bf16{h[ch]};
    };

    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int strip = u % strips, g = (u / strips) % groups, b = u / (strips * groups);
        const int j0 = strip * 64, i0 = g * WG_ROWS, i1 = min(i0 + WG_ROWS, H);
        __syncthreads();  // the previous unit's reads are done
        put(&sa[(i0 - 1 + 3) % 3][0][0], act, b, i0 - 1, j0 + lane, lane);
        put(&sa[i0 % 3][0][0], act, b, i0, j0 + lane, lane);
        for (int i = i0; i < i1; ++i) {
            __syncthreads();  // the previous row's reads are done
            put(&sa[(i + 1) % 3][0][0], act, b, i + 1, j0 + lane, lane);
            // dz row i: this lane's pixel j0 + lane goes to column lane + (c - 1) of copy c
            {
                uint4 v[4] = {make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0),
                              make_uint4(0, 0, 0, 0)};
                const int jj = j0 + lane;
                if (jj < W) {
                    const uint4 *gp = reinterpret_cast<const uint4 *>(dz + (((long long)b * H + i) * W + jj) * C);
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = gp[q];
                }
                const unsigned short *h = reinterpret_cast<const unsigned short *>(v);
#pragma unroll
                for (int ch = 0; ch < C; ++ch) {
                    if (lane >= 1) sd[0][ch][lane - 1] = bf16{h[ch]};
                    sd[1][ch][lane] = bf16{h[ch]};
                    if (lane <= 62) sd[2][ch][lane + 1] = bf16{h[ch]};
                }
            }
            // the two pixels beyond the strip: j0 + 64 -> copy 0 column 63, j0 - 1 -> copy 2 column 0
            if (lane == 0) put(&sd[2][0][0], dz, b, i, j0 - 1, 0);
            if (lane == 63) put(&sd[0][0][0], dz, b, i, j0 + 64, 63);
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int slot = (i + a - 1 + 3) % 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc) {
                        const int px0 = 16 * kc + 8 * kg;
                        bf16x8 av, bv;
                        __builtin_memcpy(&av, &sd[c][n][px0], 16);
                        __builtin_memcpy(&bv, &sa[slot][n][px0], 16);
                        acc[3 * a + c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[3 * a + c], 0, 0, 0);
                    }
                }
            }
        }
    }
    // accumulator register r of tap t: co = 8 (r / 4) + 4 kg + r % 4, ci = n
    float *dst = part + (size_t)blockIdx.x * NW2;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[((8 * (r / 4) + 4 * kg + r % 4) * C + n) * 9 + t] = acc[t][r];
}

// Weight gradients of the thin layers.  Work units of WT_ROWS image rows x 64 columns of
// one image; one wave per unit (waves beyond WT_WAVES take further units in a fixed
// stride, adding into the same slot).  Lane (c = lane mod 32, half = lane / 32) owns
// channel c and 32 of the unit's columns: along each row it slides a 3 x 3 window of the
// shifted operand (three new loads per pixel, coalesced over the 32 channel lanes or the
// same address for all), multiplies by the pixel's own operand and keeps the 9 tap sums
// in registers.  The two halves are added (lower half first) and the 288 sums of the wave
// written to its slot.
//   layer 1: part[slot][co*9 + t] = sum dz1[p][co] * a0[p + off_t]  (a0 = BF16 of x, as the
//            forward pass used)
//   layer 4: part[slot][ci*9 + t] = sum dy[p] * a3[p + off_t][ci]
template <bool L4>
__global__ __launch_bounds__(64) void wgrad_thin_kernel(const float *__restrict__ x, int ldx,
                                                        const bf16 *__restrict__ a3, const float *__restrict__ dy,
                                                        const bf16 *__restrict__ dz1, float *__restrict__ part,
                                                        int B, int H, int W)
{
    static_assert(NW1 == NW4, "one partial layout for both thin layers");
    const int strips = (W + 63) / 64, groups = (H + WT_ROWS - 1) / WT_ROWS;
    const long long units = (long long)B * groups * strips;
    const int lane = threadIdx.x, ch = lane & 31, half = lane >> 5;
    float acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = 0.0f;
    for (long long u = blockIdx.x; u < units; u += gridDim.x) {
        const int b = (int)(u / ((long long)groups * strips));
        const int rem = (int)(u % ((long long)groups * strips));
        const int i0 = (rem / strips) * WT_ROWS, i1 = min(i0 + WT_ROWS, H);
        const int j0 = (rem % strips) * 64 + half * 32, j1 = min(j0 + 32, W);
        const long long img = (long long)b * H;
        for (int i = i0; i < i1; ++i) {
            if (j0 >= j1) break;
            // the three source rows of this output row (null outside the image), so the
            // loads below index with 32-bit column offsets
            const bf16 *ra[3];
            const float *rx[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int ii = i + r - 1;
                const bool in = ii >= 0 && ii < H;
                ra[r] = (L4 && in) ? a3 + ((img + ii) * W) * C + ch : nullptr;
                rx[r] = (!L4 && in) ? x + (img + ii) * ldx : nullptr;
            }
            // shifted operand of source row r at column jj, zero outside the image
            auto sh = [&](int r, int jj) -> float {
                const bool ok = jj >= 0 && jj < W;
                if (L4) return (ra[r] && ok) ? bfv(ra[r][jj * C]) : 0.0f;
                return (rx[r] && ok) ? bf16_to_f32(f32_to_bf16_rne(rx[r][jj])) : 0.0f;
            };
            float w0[3], w1[3], w2[3];  // columns j - 1, j, j + 1 of rows i - 1, i, i + 1
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                w0[r] = sh(r, j0 - 1);
                w1[r] = sh(r, j0);
            }
            // four pixels per step: all their loads are issued before the products, so
            // a wave keeps 16 loads in flight instead of waiting on each pixel's
            for (int j = j0; j < j1; j += 4) {
                float nw[4][3], pv[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
#pragma unroll
                    for (int r = 0; r < 3; ++r) nw[e][r] = sh(r, j + e + 1);
                    const long long q = (img + i) * W + j + e;
                    pv[e] = (j + e < j1) ? (L4 ? dy[q] : bfv(dz1[q * C + ch])) : 0.0f;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        w2[r] = nw[e][r];
                        acc[3 * r] = fmaf(pv[e], w0[r], acc[3 * r]);
                        acc[3 * r + 1] = fmaf(pv[e], w1[r], acc[3 * r + 1]);
                        acc[3 * r + 2] = fmaf(pv[e], w2[r], acc[3 * r + 2]);
                        w0[r] = w1[r];
                        w1[r] = w2[r];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const float other = __shfl_down(acc[t], 32, 64);
        if (half == 0) part[(size_t)blockIdx.x * NW1 + ch * 9 + t] = acc[t] + other;
    }
}

// g[q] = sum over slots of part[slot][q], in two passes with a fixed split: slice s of
// gridDim.y adds its contiguous run of slots in order into mid[s][q]; then the slices are
// added in order.  Deterministic, and wide enough to keep the whole chip busy.
__global__ __launch_bounds__(BX) void reduce_wgrad_slices_kernel(const float *__restrict__ part, int nblk, int count,
                                                                 float *__restrict__ mid)
{
    const int q = blockIdx.x * BX + threadIdx.x;
    if (q >= count) return;
    const int ns = gridDim.y;
    const int k0 = (int)((long long)nblk * blockIdx.y / ns), k1 = (int)((long long)nblk * (blockIdx.y + 1) / ns);
    float s = 0.0f;
    for (int k = k0; k < k1; ++k) s += part[(size_t)k * count + q];
    mid[(size_t)blockIdx.y * count + q] = s;
}

__global__ __launch_bounds__(BX) void reduce_wgrad_kernel(const float *__restrict__ mid, int ns, int count,
                                                          float *__restrict__ g)
{
    const int q = blockIdx.x * BX + threadIdx.x;
    if (q >= count) return;
    float s = 0.0f;
    for (int k = 0; k < ns; ++k) s += mid[(size_t)k * count + q];
    g[q] = s;
}

__global__ __launch_bounds__(BX) void adam_kernel(float *__restrict__ w, const float *__restrict__ g,
                                                  float *__restrict__ m, float *__restrict__ v, float lr,
                                                  float b1, float b2, float eps, float c1, float c2)
{
    const int q = blockIdx.x * BX + threadIdx.x;
    if (q >= NPARAM) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    w[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// ---- pieces of the learned refinement (FP64 grids, odd reflection at the edges)

// 5-point stencil of an n x n field v (rows of ldv) at (i, j), reading only the n x n
// interior: a neighbour outside is -v(i, j).  Sum order ((((N - 4C) + W) + E) + S).
template <typename TV>
__device__ __forceinline__ double stencil_odd(const TV *__restrict__ v, int ldv, int n, int i, int j)
{
    const double c = (double)v[(long long)i * ldv + j];
    const double vn = i > 0 ? (double)v[(long long)(i - 1) * ldv + j] : -c;
    const double vs = i < n - 1 ? (double)v[(long long)(i + 1) * ldv + j] : -c;
    const double vw = j > 0 ? (double)v[(long long)i * ldv + j - 1] : -c;
    const double ve = j < n - 1 ? (double)v[(long long)i * ldv + j + 1] : -c;
    return (((vn - 4.0 * c) + vw) + ve) + vs;
}

// Pair, first pass over phi's interior (phi + ld + 1 is cell (1, 1)): per-block partial
// sums {S(phi)^2, e^2 or e K e} with e = -phi and K e = -S(e) = S(phi).
__global__ __launch_bounds__(BX) void pair_sums_kernel(const double *__restrict__ phi, int n, int ld, int loss,
                                                       double2 *__restrict__ part)
{
    __shared__ double sh[BX];
    const int i = blockIdx.y, j = blockIdx.x * BX + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (j < n) {
        const double *in = phi + ld + 1;
        const double sp = stencil_odd(in, ld, n, i, j);
        const double e = -in[(long long)i * ld + j];
        a = sp * sp;
        b = loss == 1 ? e * sp : e * e;
    }
    const double ta = block_sum(a, sh);
    __syncthreads();
    const double tb = block_sum(b, sh);
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = make_double2(ta, tb);
}

// Pair, second pass: x = -S(phi) / sqrt(sums[0] / n^2), t = -phi / sqrt(sums[1] / n^2).
__global__ __launch_bounds__(BX) void pair_write_kernel(const double *__restrict__ phi, int n, int ld,
                                                        const double *__restrict__ sums, float *__restrict__ x,
                                                        float *__restrict__ t)
{
    const int i = blockIdx.y, j = blockIdx.x * BX + threadIdx.x;
    if (j >= n) return;
    const double cells = (double)n * (double)n;
    const double rx = sqrt(sums[0] / cells), rt = sqrt(sums[1] / cells);
    const double *in = phi + ld + 1;
    const double sp = stencil_odd(in, ld, n, i, j);
    x[(long long)i * n + j] = rx > 0.0 ? (float)(-sp / rx) : 0.0f;
    t[(long long)i * n + j] = rt > 0.0 ? (float)(-in[(long long)i * ld + j] / rt) : 0.0f;
}

// Per-block partial sums of the correction step over the n x n interior:
// {<r, r>, <d, r>, <r, S r>, <r, S d>, <d, S d>} (S with odd reflection; S is symmetric,
// so <d, S r> = <r, S d>).  part: 8 doubles per block.
template <typename TD>
__global__ __launch_bounds__(BX) void dots_kernel(const TD *__restrict__ d, int ld_d, const double *__restrict__ r,
                                                  int ld_r, int n, double *__restrict__ part)
{
    __shared__ double sh[BX];
    const int i = blockIdx.y, j = blockIdx.x * BX + threadIdx.x;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (j < n) {
        const double rv = r[(long long)i * ld_r + j], dv = (double)d[(long long)i * ld_d + j];
        const double sr = stencil_odd(r, ld_r, n, i, j), sd = stencil_odd(d, ld_d, n, i, j);
        v[0] = rv * rv;
        v[1] = dv * rv;
        v[2] = rv * sr;
        v[3] = rv * sd;
        v[4] = dv * sd;
    }
    double *dst = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 8;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const double t = block_sum(v[q], sh);
        if (threadIdx.x == 0) dst[q] = t;
        __syncthreads();
    }
}

// out[q] = sum over blocks (fixed order) of part[blk * 8 + q], q = 0..4.
__global__ __launch_bounds__(BX) void sum5_partials_kernel(const double *__restrict__ part, int count,
                                                           double *__restrict__ out)
{
    __shared__ double sh[BX];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        double s = 0.0;
        for (int k = threadIdx.x; k < count; k += BX) s = s + part[(size_t)k * 8 + q];
        const double t = block_sum(s, sh);
        if (threadIdx.x == 0) out[q] = t;
        __syncthreads();
    }
}

// Coefficients (a, b) of phi += a r + b d that minimise the energy norm of the error
// e (L e = r, L = c S) over the allowed directions: the Galerkin conditions
// <v, L(a r + b d)> = <v, r> for v in the span, i.e. c M (a, b) = (<r,r>, <d,r>) with
// M = [<r,Sr> <r,Sd>; <r,Sd> <d,Sd>].  mode 0: r only; 1: d only; 2: both (r only if
// M is numerically singular).  A zero denominator gives a zero step.
__device__ __forceinline__ void step_coefficients(const double *dots, double c, int mode, double &a, double &b)
{
    const double rr = dots[0], dr = dots[1], rsr = dots[2], rsd = dots[3], dsd = dots[4];
    a = 0.0;
    b = 0.0;
    if (mode == 2) {
        const double det = rsr * dsd - rsd * rsd;
        if (fabs(det) > 1e-10 * fabs(rsr * dsd)) {
            a = (rr * dsd - rsd * dr) / (c * det);
            b = (rsr * dr - rsd * rr) / (c * det);
            return;
        }
        mode = 0;
    }
    if (mode == 0) a = rsr != 0.0 ? rr / (c * rsr) : 0.0;
    else b = dsd != 0.0 ? dr / (c * dsd) : 0.0;
}

// phi(i, j) += a r(i, j) + b d(i, j) over the interior; coef (if not NULL) gets (a, b).
template <typename TD>
__global__ __launch_bounds__(BX) void step_kernel(const TD *__restrict__ d, int ld_d, const double *__restrict__ r,
                                                  int ld_r, double *__restrict__ phi, int n, int ld, double c,
                                                  const double *__restrict__ dots, int mode, double *__restrict__ coef)
{
    const int i = blockIdx.y, j = blockIdx.x * BX + threadIdx.x;
    double a, b;
    step_coefficients(dots, c, mode, a, b);
    if (coef && i == 0 && j == 0) {
        coef[0] = a;
        coef[1] = b;
    }
    if (j >= n) return;
    double *p = phi + (long long)(i + 1) * ld + (j + 1);
    *p = (*p + a * r[(long long)i * ld_r + j]) + b * (double)d[(long long)i * ld_d + j];
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + BX - 1) / BX); }

// ---- network state

struct NetState {
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    bf16 *wb = nullptr;  // all BF16 layouts in one allocation
    NetW nw{};
    long long pixels = 0;  // workspace capacity
    bf16 *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *dz1 = nullptr, *dz2 = nullptr, *dz3 = nullptr;
    float *y = nullptr, *dy = nullptr, *part = nullptr, *mid = nullptr;
    double *dpart = nullptr;
    long long step = 0;
    long long last_pixels = 0;  // pixels of the last forward pass (0: none yet)

    void free_workspace()
    {
        for (bf16 **p : {&a1, &a2, &a3, &dz1, &dz2, &dz3}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        for (float **p : {&y, &dy}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        if (dpart) (void)hipFree(dpart);
        dpart = nullptr;
        pixels = 0;
    }
    ~NetState()
    {
        free_workspace();
        for (float **p : {&w, &m, &v, &g, &part, &mid}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        if (wb) (void)hipFree(wb);
    }
};

hipError_t net_alloc(NetState &s)
{
    hipError_t e;
    for (float **p : {&s.w, &s.m, &s.v, &s.g})
        if ((e = hipMalloc(p, sizeof(float) * NPARAM)) != hipSuccess) return e;
    if ((e = hipMalloc(&s.wb, sizeof(bf16) * (NW1 + 4 * NW2 + NW4))) != hipSuccess) return e;
    s.nw.w1 = s.wb;
    s.nw.w2f = s.wb + NW1;
    s.nw.w2b = s.nw.w2f + NW2;
    s.nw.w3f = s.nw.w2b + NW2;
    s.nw.w3b = s.nw.w3f + NW2;
    s.nw.w4 = s.nw.w3b + NW2;
    static_assert((size_t)WT_WAVES * NW1 <= (size_t)WGM_BLOCKS * NW2, "thin partials fit the partial buffer");
    if ((e = hipMalloc(&s.mid, sizeof(float) * (size_t)RS * NW2)) != hipSuccess) return e;
    return hipMalloc(&s.part, sizeof(float) * (size_t)WGM_BLOCKS * NW2);
}

hipError_t net_set(NetState &s, const float *host)
{
    hipError_t e;
    if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
    if ((e = hipMemcpy(s.w, host, sizeof(float) * NPARAM, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemset(s.m, 0, sizeof(float) * NPARAM)) != hipSuccess) return e;
    if ((e = hipMemset(s.v, 0, sizeof(float) * NPARAM)) != hipSuccess) return e;
    if ((e = hipMemset(s.g, 0, sizeof(float) * NPARAM)) != hipSuccess) return e;
    s.step = 0;
    hipLaunchKernelGGL(prep_weights_kernel, dim3(blocks_for(NPARAM)), dim3(BX), 0, 0, s.w, s.nw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipDeviceSynchronize();
}

hipError_t net_workspace(NetState &s, long long pixels)
{
    if (pixels <= s.pixels) return hipSuccess;
    hipError_t e;
    if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
    s.free_workspace();
    for (bf16 **p : {&s.a1, &s.a2, &s.a3, &s.dz1, &s.dz2, &s.dz3})
        if ((e = hipMalloc(p, sizeof(bf16) * C * (size_t)pixels)) != hipSuccess) return e;
    for (float **p : {&s.y, &s.dy})
        if ((e = hipMalloc(p, sizeof(float) * (size_t)pixels)) != hipSuccess) return e;
    if ((e = hipMalloc(&s.dpart, sizeof(double) * blocks_for(pixels))) != hipSuccess) return e;
    s.pixels = pixels;
    return hipSuccess;
}

unsigned conv_blocks(int B, int H, int W)
{
    const long long tiles = (long long)B * ((H + TROWS - 1) / TROWS) * ((W + TPX - 1) / TPX);
    return (unsigned)std::min<long long>(tiles, 2048);  // 8 blocks per CU; blocks loop over tiles
}

unsigned thin_blocks(int B, int H, int W)
{
    return (unsigned)((long long)B * ((H + LT_ROWS - 1) / LT_ROWS) * ((W + LT_PX - 1) / LT_PX));
}

// Forward pass: y (rows of ldy) = N(x * scale); x rows of ldx, FP64 or FP32.
hipError_t net_forward(NetState &s, int xdt, const void *x, int ldx, double scale, float *y, int ldy, int B, int H,
                       int W, hipStream_t st)
{
    const long long N = (long long)B * H * W;
    hipError_t e = net_workspace(s, N);
    if (e != hipSuccess) return e;
    const unsigned lt = thin_blocks(B, H, W);
    if (xdt == F64)
        hipLaunchKernelGGL(l1_fwd_kernel<double>, dim3(lt), dim3(BX), 0, st, (const double *)x, ldx, scale, s.nw.w1,
                           s.a1, B, H, W);
    else
        hipLaunchKernelGGL(l1_fwd_kernel<float>, dim3(lt), dim3(BX), 0, st, (const float *)x, ldx, scale, s.nw.w1,
                           s.a1, B, H, W);
    hipLaunchKernelGGL(conv32_kernel<false>, dim3(conv_blocks(B, H, W)), dim3(BX), 0, st, s.a1, s.nw.w2f, s.a2,
                       (const bf16 *)nullptr, B, H, W);
    hipLaunchKernelGGL(conv32_kernel<false>, dim3(conv_blocks(B, H, W)), dim3(BX), 0, st, s.a2, s.nw.w3f, s.a3,
                       (const bf16 *)nullptr, B, H, W);
    hipLaunchKernelGGL(l4_fwd_kernel, dim3(conv_blocks(B, H, W)), dim3(BX), 0, st, s.a3, s.nw.w4, y, ldy, B, H, W);
    s.last_pixels = N;
    return hipGetLastError();
}

// Inference: y = N(x * scale) as net_forward computes it, layers 1 and 2 fused (conv12_kernel),
// so the layer-1 activations never reach memory; the hidden activations are not kept.
hipError_t net_infer_forward(NetState &s, int xdt, const void *x, int ldx, double scale, float *y, int ldy, int B,
                             int H, int W, hipStream_t st)
{
    const long long N = (long long)B * H * W;
    hipError_t e = net_workspace(s, N);
    if (e != hipSuccess) return e;
    const unsigned cb = conv_blocks(B, H, W);
    if (xdt == F64)
        hipLaunchKernelGGL(conv12_kernel<double>, dim3(cb), dim3(BX), 0, st, (const double *)x, ldx, scale, s.nw.w1,
                           s.nw.w2f, s.a2, B, H, W);
    else
        hipLaunchKernelGGL(conv12_kernel<float>, dim3(cb), dim3(BX), 0, st, (const float *)x, ldx, scale, s.nw.w1,
                           s.nw.w2f, s.a2, B, H, W);
    hipLaunchKernelGGL(conv32_kernel<false>, dim3(cb), dim3(BX), 0, st, s.a2, s.nw.w3f, s.a3, (const bf16 *)nullptr,
                       B, H, W);
    hipLaunchKernelGGL(l4_fwd_kernel, dim3(cb), dim3(BX), 0, st, s.a3, s.nw.w4, y, ldy, B, H, W);
    s.last_pixels = 0;  // the layer-1 activations of this pass were never stored
    return hipGetLastError();
}

// Forward, loss and backward on compact FP32 x and t; gradient into s.g, loss into *loss.
hipError_t net_gradient(NetState &s, const float *x, const float *t, int B, int H, int W, int loss,
                        double *loss_out, hipStream_t st)
{
    const long long N = (long long)B * H * W;
    hipError_t e = net_workspace(s, N);
    if (e != hipSuccess) return e;
    if ((e = net_forward(s, F32, x, W, 1.0, s.y, W, B, H, W, st)) != hipSuccess) return e;
    if (loss == 0) {
        hipLaunchKernelGGL(mse_kernel, dim3(blocks_for(N)), dim3(BX), 0, st, s.y, t, s.dy, s.dpart, N);
    } else {
        hipLaunchKernelGGL(diff_kernel, dim3(blocks_for(N)), dim3(BX), 0, st, s.y, t, N);
        hipLaunchKernelGGL(energy_kernel, dim3(blocks_for(N)), dim3(BX), 0, st, s.y, s.dy, s.dpart, B, H, W);
    }
    if (loss_out)
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(BX), 0, st, s.dpart, (int)blocks_for(N), loss_out,
                           1.0 / (double)N);
    const unsigned cb = conv_blocks(B, H, W);
    const unsigned wgm = (unsigned)std::min<long long>(
        (long long)B * ((W + 63) / 64) * ((H + WG_ROWS - 1) / WG_ROWS), WGM_BLOCKS);
    const unsigned wtn = (unsigned)std::min<long long>(
        (long long)B * ((W + 63) / 64) * ((H + WT_ROWS - 1) / WT_ROWS), WT_WAVES);
    auto reduce = [&](unsigned nblk, int count, float *g) {
        const int ns = count == NW2 ? RS : RS_THIN;
        hipLaunchKernelGGL(reduce_wgrad_slices_kernel, dim3(blocks_for(count), ns), dim3(BX), 0, st, s.part,
                           (int)nblk, count, s.mid);
        hipLaunchKernelGGL(reduce_wgrad_kernel, dim3(blocks_for(count)), dim3(BX), 0, st, s.mid, ns, count, g);
    };
    // layer 4
    hipLaunchKernelGGL(wgrad_thin_kernel<true>, dim3(wtn), dim3(64), 0, st, (const float *)nullptr, 0, s.a3, s.dy,
                       (const bf16 *)nullptr, s.part, B, H, W);
    reduce(wtn, NW4, s.g + OFF4);
    hipLaunchKernelGGL(l4_bwd_kernel, dim3(blocks_for(N)), dim3(BX), 0, st, s.dy, s.nw.w4, s.a3, s.dz3, B, H, W);
    // layer 3
    hipLaunchKernelGGL(wgrad32_mfma_kernel, dim3(wgm), dim3(64), 0, st, s.a2, s.dz3, s.part, B, H, W);
    reduce(wgm, NW2, s.g + OFF3);
    hipLaunchKernelGGL(conv32_kernel<true>, dim3(cb), dim3(BX), 0, st, s.dz3, s.nw.w3b, s.dz2, s.a2, B, H, W);
    // layer 2
    hipLaunchKernelGGL(wgrad32_mfma_kernel, dim3(wgm), dim3(64), 0, st, s.a1, s.dz2, s.part, B, H, W);
    reduce(wgm, NW2, s.g + OFF2);
    hipLaunchKernelGGL(conv32_kernel<true>, dim3(cb), dim3(BX), 0, st, s.dz2, s.nw.w2b, s.dz1, s.a1, B, H, W);
    // layer 1
    hipLaunchKernelGGL(wgrad_thin_kernel<false>, dim3(wtn), dim3(64), 0, st, x, W, (const bf16 *)nullptr,
                       (const float *)nullptr, s.dz1, s.part, B, H, W);
    reduce(wtn, NW1, s.g);
    return hipGetLastError();
}

hipError_t net_adam(NetState &s, float lr, hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    s.step += 1;
    const float c1 = 1.0f - std::pow(b1, (float)s.step), c2 = 1.0f - std::pow(b2, (float)s.step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(NPARAM)), dim3(BX), 0, st, s.w, s.g, s.m, s.v, lr, b1, b2, eps,
                       c1, c2);
    hipLaunchKernelGGL(prep_weights_kernel, dim3(blocks_for(NPARAM)), dim3(BX), 0, st, s.w, s.nw);
    return hipGetLastError();
}

}  // namespace

int pair_num_blocks(int n) { return (int)blocks_for(n) * n; }

hipError_t pair_launch(const double *phi, int n, int ld, int loss, float *x, float *t, double *part, double *sums,
                       hipStream_t s)
{
    const dim3 grid(blocks_for(n), n);
    hipLaunchKernelGGL(pair_sums_kernel, grid, dim3(BX), 0, s, phi, n, ld, loss, (double2 *)part);
    hipLaunchKernelGGL(sum2_partials_kernel, dim3(1), dim3(BX), 0, s, (const double2 *)part, pair_num_blocks(n),
                       sums);
    hipLaunchKernelGGL(pair_write_kernel, grid, dim3(BX), 0, s, phi, n, ld, (const double *)sums, x, t);
    return hipGetLastError();
}

hipError_t correction_launch(int ddtype, const void *d, int ld_d, const double *r, int ld_r, double *phi, int n,
                             int ld, double c, int mode, double *part, double *dots, double *coef, hipStream_t s)
{
    const dim3 grid(blocks_for(n), n);
    if (ddtype == F64)
        hipLaunchKernelGGL(dots_kernel<double>, grid, dim3(BX), 0, s, (const double *)d, ld_d, r, ld_r, n, part);
    else
        hipLaunchKernelGGL(dots_kernel<float>, grid, dim3(BX), 0, s, (const float *)d, ld_d, r, ld_r, n, part);
    hipLaunchKernelGGL(sum5_partials_kernel, dim3(1), dim3(BX), 0, s, (const double *)part, pair_num_blocks(n), dots);
    if (ddtype == F64)
        hipLaunchKernelGGL(step_kernel<double>, grid, dim3(BX), 0, s, (const double *)d, ld_d, r, ld_r, phi, n, ld, c,
                           (const double *)dots, mode, coef);
    else
        hipLaunchKernelGGL(step_kernel<float>, grid, dim3(BX), 0, s, (const float *)d, ld_d, r, ld_r, phi, n, ld, c,
                           (const double *)dots, mode, coef);
    return hipGetLastError();
}

}  // namespace px

// ------------------------------------------------------------------ ABI

struct px_net {
    int device = 0;
    px::NetState s;
};

namespace px {

hipError_t net_infer(px_net *net, const double *r, int ld_r, int n, double scale, float *y, int ld_y, hipStream_t s)
{
    return net_infer_forward(net->s, F64, r, ld_r, scale, y, ld_y, 1, n, n, s);
}

int net_device(const px_net *net) { return net->device; }

}  // namespace px

using px::set_error;

namespace {

constexpr long long MAX_PIXELS = 1LL << 31;

int hip_err(hipError_t e, const char *what) { return set_error(PX_EHIP, "%s: %s", what, hipGetErrorString(e)); }

int check_images(int batch, int H, int W)
{
    if (batch < 1 || H < 1 || W < 1) return set_error(PX_EINVAL, "batch, H and W must be >= 1");
    if ((long long)batch * H * W > MAX_PIXELS) return set_error(PX_EINVAL, "more than 2^31 pixels");
    return PX_OK;
}

int use_device(const px_net *net)
{
    hipError_t e = hipSetDevice(net->device);
    return e == hipSuccess ? PX_OK : hip_err(e, "hipSetDevice");
}

}  // namespace

extern "C" {

int px_net_create(int device, const float *weights, px_net **out)
{
    if (!out) return set_error(PX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!weights) return set_error(PX_EINVAL, "weights is NULL");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_err(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return set_error(PX_EINVAL, "device %d not present", device);
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_err(e, "hipSetDevice");
    px_net *net = new (std::nothrow) px_net;
    if (!net) return set_error(PX_ENOMEM, "out of host memory");
    net->device = device;
    if ((e = px::net_alloc(net->s)) != hipSuccess || (e = px::net_set(net->s, weights)) != hipSuccess) {
        delete net;
        return e == hipErrorOutOfMemory ? set_error(PX_ENOMEM, "network allocation failed") : hip_err(e, "network set-up");
    }
    *out = net;
    return PX_OK;
}

int px_net_destroy(px_net *net)
{
    if (!net) return PX_OK;
    int st = use_device(net);
    if (st) return st;
    (void)hipDeviceSynchronize();
    delete net;
    return PX_OK;
}

int px_net_set_weights(px_net *net, const float *weights)
{
    if (!net || !weights) return set_error(PX_EINVAL, "net or weights is NULL");
    int st = use_device(net);
    if (st) return st;
    hipError_t e = px::net_set(net->s, weights);
    return e == hipSuccess ? PX_OK : hip_err(e, "px_net_set_weights");
}

int px_net_get_weights(px_net *net, float *weights)
{
    if (!net || !weights) return set_error(PX_EINVAL, "net or weights is NULL");
    int st = use_device(net);
    if (st) return st;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(weights, net->s.w, sizeof(float) * px::NPARAM, hipMemcpyDeviceToHost);
    return e == hipSuccess ? PX_OK : hip_err(e, "px_net_get_weights");
}

int px_net_forward(px_net *net, const void *x, int x_dtype, int ldx, int batch, int H, int W, double x_scale,
                   float *y, int ldy, void *stream)
{
    if (!net || !x || !y) return set_error(PX_EINVAL, "net, x or y is NULL");
    if (x_dtype != PX_F64 && x_dtype != PX_F32) return set_error(PX_EINVAL, "x_dtype must be PX_F64 or PX_F32");
    int st = check_images(batch, H, W);
    if (st) return st;
    if (ldx < W || ldy < W) return set_error(PX_EINVAL, "ldx and ldy must be >= W");
    if (!std::isfinite(x_scale)) return set_error(PX_EINVAL, "x_scale must be finite");
    if ((st = use_device(net))) return st;
    hipError_t e = px::net_forward(net->s, x_dtype, x, ldx, x_scale, y, ldy, batch, H, W, (hipStream_t)stream);
    if (e == hipErrorOutOfMemory) return set_error(PX_ENOMEM, "network workspace allocation failed");
    return e == hipSuccess ? PX_OK : hip_err(e, "network forward launch");
}

int px_net_loss_grad(px_net *net, const float *x, const float *t, int batch, int H, int W, int loss,
                     double *loss_out, float *grad, void *stream)
{
    if (!net || !x || !t) return set_error(PX_EINVAL, "net, x or t is NULL");
    if (loss != PX_LOSS_MSE && loss != PX_LOSS_ENERGY) return set_error(PX_EINVAL, "unknown loss %d", loss);
    int st = check_images(batch, H, W);
    if (st) return st;
    if ((st = use_device(net))) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = px::net_gradient(net->s, x, t, batch, H, W, loss, loss_out, s);
    if (e == hipSuccess && grad)
        e = hipMemcpyAsync(grad, net->s.g, sizeof(float) * px::NPARAM, hipMemcpyDeviceToDevice, s);
    if (e == hipErrorOutOfMemory) return set_error(PX_ENOMEM, "network workspace allocation failed");
    return e == hipSuccess ? PX_OK : hip_err(e, "network gradient launch");
}

int px_net_adam(px_net *net, float lr, void *stream)
{
    if (!net) return set_error(PX_EINVAL, "net is NULL");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return set_error(PX_EINVAL, "lr must be finite and > 0");
    int st = use_device(net);
    if (st) return st;
    hipError_t e = px::net_adam(net->s, lr, (hipStream_t)stream);
    return e == hipSuccess ? PX_OK : hip_err(e, "Adam launch");
}

int px_net_infer(px_net *net, const void *x, int x_dtype, int ldx, int batch, int H, int W, double x_scale, float *y,
                 int ldy, void *stream)
{
    if (!net || !x || !y) return set_error(PX_EINVAL, "net, x or y is NULL");
    if (x_dtype != PX_F64 && x_dtype != PX_F32) return set_error(PX_EINVAL, "x_dtype must be PX_F64 or PX_F32");
    int st = check_images(batch, H, W);
    if (st) return st;
    if (ldx < W || ldy < W) return set_error(PX_EINVAL, "ldx and ldy must be >= W");
    if (!std::isfinite(x_scale)) return set_error(PX_EINVAL, "x_scale must be finite");
    if ((st = use_device(net))) return st;
    hipError_t e = px::net_infer_forward(net->s, x_dtype, x, ldx, x_scale, y, ldy, batch, H, W, (hipStream_t)stream);
    if (e == hipErrorOutOfMemory) return set_error(PX_ENOMEM, "network workspace allocation failed");
    return e == hipSuccess ? PX_OK : hip_err(e, "network inference launch");
}

int px_net_activation(px_net *net, int layer, uint16_t *out, void *stream)
{
    if (!net || !out) return set_error(PX_EINVAL, "net or out is NULL");
    if (layer < 1 || layer > 3) return set_error(PX_EINVAL, "layer must be 1, 2 or 3");
    if (net->s.last_pixels == 0) return set_error(PX_EINVAL, "no forward pass yet");
    int st = use_device(net);
    if (st) return st;
    const px::bf16 *a = layer == 1 ? net->s.a1 : layer == 2 ? net->s.a2 : net->s.a3;
    hipError_t e = hipMemcpyAsync(out, a, sizeof(px::bf16) * px::C * (size_t)net->s.last_pixels,
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? PX_OK : hip_err(e, "activation copy");
}

}  // extern "C"
