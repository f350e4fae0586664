// Learned preconditioner of the Anderson step: a 4-layer 3x3 CNN
// (channels 2 -> 32 -> 32 -> 32 -> 1, ReLU after the first three, zero "same"
// padding, no bias) on bf16 activations and weights with FP32 accumulation on
// the matrix cores, its hand-written backward, the scale-free loss and Adam.
//
// The network maps [g / rms(g), (m - mean m) / std m] of one image to z; the
// search direction is d = softplus(z) * g, so d = 0 exactly when g = 0 (the
// fixed points of the descent map G of eq. GD are kept) and <d, g> > 0.
// Training target for a step s taken by an optimiser: t = -s / rms(s); loss
// per image mean((d / rms(d) - t)^2), averaged over the batch.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16: one wave owns
// 16 consecutive pixels and all output channels (16-channel tiles); the
// reduction runs over (tap, channel) in chunks of 32.
// Activations are NHWC with the channel count padded to 16 or 32.
// Weight copies: Wf[tap][co][ci] (forward), Wd[tap][ci][co] (input gradient).
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "common.hpp"

namespace aafwi {
namespace {

typedef unsigned short bf16;
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kL = 4;
constexpr int kCinP[kL] = {16, 32, 32, 32};   // padded input channels
constexpr int kCoutP[kL] = {32, 32, 32, 16};  // padded output channels
constexpr int kCin[kL] = {2, 32, 32, 32};
constexpr int kCout[kL] = {32, 32, 32, 1};
constexpr int kRedBlocks = 64;     // per-image reduction partials

__device__ __forceinline__ bf16 f2bf(float f) {
    unsigned u = __builtin_bit_cast(unsigned, f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 h) { return __builtin_bit_cast(float, (unsigned)h << 16); }

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf8 ld8(const bf16* p) { return __builtin_bit_cast(bf8, *reinterpret_cast<const v4u*>(p)); }
__device__ __forceinline__ bf8 zero8() { return __builtin_bit_cast(bf8, v4u{0u, 0u, 0u, 0u}); }

enum ConvMode { kHidden = 0, kLast = 1, kInputGrad = 2 };

// 3x3 convolution as an implicit GEMM on v_mfma_f32_16x16x32_bf16, for the
// forward pass (x: [P][C] -> y: [P][NOUT] with ReLU, or z: [P] FP32 for the
// last layer) and the input gradient (x = dy: [P][C], taps mirrored, output
// masked by the ReLU of the layer input `mask`).  The reduction index is
// k = tap * C + c, cut into chunks of 32: lane group g of a fragment holds
// k = 32 ch + 8 g .. 8 g + 7, i.e. 8 consecutive channels of one tap.  w is
// [tap][NOUT][C] bf16; every wave keeps all its weight fragments in
// registers.  A block of four waves owns a 64-pixel-wide column segment of
// one image over a run of rows and walks down it two output rows per pass:
// an LDS ring of six row slots holds input rows y-1 .. y+2 (columns x0-1 ..
// x0+64, zeros outside the image), each pass adds two new input rows, and the
// two after those are fetched into registers while the current pair runs on
// the matrix cores (four independent accumulation chains per wave).  The
// rows being written are never among the four being read, so one barrier per
// pass orders the two.  Wave w takes pixels x0+16w .. x0+16w+15 and reads
// each activation fragment as one 16-byte LDS load.  For the 32-channel
// outputs the weights are the A operand and the activations the B operand,
// so a lane's accumulators hold four consecutive channels of one pixel and
// go to HBM as 8-byte stores; the 16-channel last layer keeps the pixels in
// the A operand (its single useful channel is then one lane group).
constexpr int kCSeg = 64;
constexpr int kConvSlots = 6;  // LDS ring of staged input rows

template <int C>
struct RowFetch {
    static constexpr int kChunks = (kCSeg + 2) * (C / 8);  // 16-byte pieces of one staged row
    static constexpr int kPer = (kChunks + 255) / 256;
    v4u v[kPer];
};

// One image of an NHWC bf16 tensor as a raw buffer resource (base in SGPRs,
// 32-bit byte offsets); the hardware range check returns zeros for loads at
// offsets at or beyond the image, which is how pieces outside the image are
// read (offset kOut).
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr unsigned kOut = 0x80000000u;
template <int C>
__device__ __forceinline__ Rsrc image_view(const bf16* x, int bimg, int H, int W) {
    const long long n = (long long)H * W * C;
    return __builtin_amdgcn_make_buffer_rsrc((void*)(x + bimg * n), (short)0, (int)(n * 2), 0x00020000);
}

// Global -> registers: input row yy over columns x0-1 .. x0+64 (zeros outside;
// a row the caller will not store, need = false, reads zeros too).  No
// branch surrounds a load and the data goes to LDS unchanged, so the
// compiler can wait for each row by count while the rows fetched after it
// stay in flight.
template <int C>
__device__ __forceinline__ void row_fetch(RowFetch<C>& f, Rsrc r, int H, int W, int yy, int x0, bool need = true) {
#pragma unroll
    for (int k = 0; k < RowFetch<C>::kPer; ++k) {
        const int e = threadIdx.x + 256 * k;
        const int cg = e % (C / 8), j = e / (C / 8);
        const int xx = x0 - 1 + j;
        const bool in = need && e < RowFetch<C>::kChunks && yy >= 0 && yy < H && xx >= 0 && xx < W;
        const unsigned off = in ? (unsigned)(((yy * W + xx) * C + cg * 8) * 2) : kOut;
        f.v[k] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    }
}

// Registers -> LDS row (pixel stride CS).
template <int C, int CS>
__device__ __forceinline__ void row_store(const RowFetch<C>& f, bf16* row) {
#pragma unroll
    for (int k = 0; k < RowFetch<C>::kPer; ++k) {
        const int e = threadIdx.x + 256 * k;
        const int cg = e % (C / 8), j = e / (C / 8);
        if (e < RowFetch<C>::kChunks) *reinterpret_cast<v4u*>(row + j * CS + cg * 8) = f.v[k];
    }
}

// The weight fragments are loaded before a kernel's main loop.  An empty asm
// statement that takes all of them as operands makes the compiler wait for
// those loads there, once, so that the loop's own waits count only the
// loads the loop issues (otherwise the first use of each fragment inside the
// loop carries a wait that also drains the rows prefetched for later passes).
template <int N, int NT>
__device__ __forceinline__ void settle(const bf8 (&bw)[N][NT]) {
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) asm volatile("" ::"v"(bw[a][b]));
}

// Products of one pass for 32 input channels (one tap per 32-wide chunk):
// two output rows from the four staged rows at base[0..3] (input rows y-1 ..
// y+2 of the first output row y).  Each (input row, column shift) fragment
// is read from LDS once and feeds both output rows that use it; every
// accumulator still takes its nine taps in ascending tap order, so the sums
// are those of a plain per-row loop over the taps.  SGN = -1 mirrors the
// taps (input gradient).  TR puts the weights in the A operand: the
// accumulators then hold four consecutive output channels of one pixel.
template <int CS, int NT, int SGN, bool TR>
__device__ __forceinline__ void conv_pass32(const bf16* L, const int (&base)[4], int aofs, const bf8 (&bw)[9][NT],
                                            v4f (&acc)[2][NT]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int s = SGN > 0 ? u : 3 - u;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const int cx = SGN > 0 ? v : 2 - v;
            const bf8 a = __builtin_bit_cast(bf8, *reinterpret_cast<const v4u*>(L + base[s] + cx * CS + aofs));
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = s - h;  // input row of this output row, relative to the row above it
                if (r < 0 || r > 2) continue;
                const int t = SGN > 0 ? 3 * r + cx : 3 * (2 - r) + (2 - cx);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[h][nt] = TR ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[t][nt], a, acc[h][nt], 0, 0, 0)
                                    : __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[t][nt], acc[h][nt], 0, 0, 0);
            }
        }
    }
}

// Four FP32 values -> four packed bf16 (8 bytes), ReLU first when asked.
__device__ __forceinline__ uint2 pack4(const v4f& a, bool relu) {
    unsigned h[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) h[q] = f2bf(relu ? fmaxf(a[q], 0.f) : a[q]);
    return uint2{h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
}

// Keep each bf16 of v where the matching bf16 of the ReLU output m is > 0.
__device__ __forceinline__ uint2 relu_mask(uint2 v, uint2 m) {
    const unsigned mm[2] = {m.x, m.y};
    unsigned keep[2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
        keep[q] = (bf2f((bf16)(mm[q] & 0xffffu)) > 0.f ? 0xffffu : 0u) | (bf2f((bf16)(mm[q] >> 16)) > 0.f ? 0xffff0000u : 0u);
    return uint2{v.x & keep[0], v.y & keep[1]};
}

template <int C, int NOUT, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_conv_mm(int B, int H, int W, int rows, const bf16* __restrict__ x,
                                                 const bf16* __restrict__ w, const bf16* __restrict__ mask,
                                                 bf16* __restrict__ y, float* __restrict__ z) {
    constexpr int NCH = (9 * C + 31) / 32;
    constexpr int NT = NOUT / 16;
    constexpr int sgn = MODE == kInputGrad ? -1 : 1;
    constexpr int CS = C + 8;                // LDS pixel stride: 16-byte aligned rows of channels
    constexpr int RW = (kCSeg + 2) * CS;     // one staged row
    static_assert(MODE == kLast || NOUT == 32, "hidden and input-gradient layers have 32 outputs");
    // 32-channel outputs: weights in the A operand, so that a lane ends with
    // four consecutive channels of its own pixel (one 8-byte store per tile)
    constexpr bool TR = MODE != kLast;
    __shared__ __align__(16) bf16 xL[kConvSlots * RW];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = lane & 15, grp = lane >> 4;
    bf8 bw[NCH][NT];
    int rsel[NCH];  // input row of this lane's A fragment relative to the output row, + 1
    int cofs[NCH];  // element offset inside a staged row, relative to the pixel
    bool tap_ok[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int k0 = 32 * ch + 8 * grp;
        const int tap = k0 / C, c0 = k0 % C;
        tap_ok[ch] = tap < 9;
        const int dyo = sgn * (tap / 3 - 1), dxo = sgn * (tap % 3 - 1);
        rsel[ch] = dyo + 1;
        cofs[ch] = (1 + dxo) * CS + c0;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            bw[ch][nt] = tap_ok[ch] ? ld8(w + ((tap * NOUT + nt * 16 + i) * C + c0)) : zero8();
    }
    settle(bw);
    auto slot = [](int r) { return ((r + kConvSlots) % kConvSlots) * RW; };  // r >= -1
    const int segs_x = (W + kCSeg - 1) / kCSeg;
    const int runs = (H + rows - 1) / rows;
    const int nwork = B * runs * segs_x;
    const int px = 16 * wv + i;  // this lane's pixel in the segment (A rows, or B columns with TR)
    for (int wk = blockIdx.x; wk < nwork; wk += gridDim.x) {
        const int sx = wk % segs_x, t = wk / segs_x;
        const int run = t % runs, bimg = t / runs;
        const int x0 = sx * kCSeg, ya = run * rows, yb = min(H, ya + rows);
        // the rows of the next two passes are in flight in registers: the
        // passes alternate between two buffer pairs; a pass stores its pair
        // (rows yy+1, yy+2) into the ring and refills it with the rows of the
        // pass after next
        const Rsrc xr = image_view<C>(x, bimg, H, W);
        RowFetch<C> fa0, fa1, fc0, fc1;
        __syncthreads();  // the ring's previous contents are no longer read
        row_fetch<C>(fc0, xr, H, W, ya - 1, x0);
        row_fetch<C>(fc1, xr, H, W, ya, x0);
        row_fetch<C>(fa0, xr, H, W, ya + 1, x0);
        row_fetch<C>(fa1, xr, H, W, ya + 2, x0);
        row_store<C, CS>(fc0, xL + slot(ya - 1));
        row_store<C, CS>(fc1, xL + slot(ya));
        row_fetch<C>(fc0, xr, H, W, ya + 3, x0, ya + 2 < yb);
        row_fetch<C>(fc1, xr, H, W, ya + 4, x0, ya + 2 < yb);
        // two output rows (yy, yy+1) per pass: input rows yy-1 .. yy+2 are
        // read; rows yy+1, yy+2 are stored at the start of the pass into the
        // slots of rows yy-5, yy-4, which the previous pass no longer reads
        auto pass = [&](int yy, RowFetch<C>& f0, RowFetch<C>& f1) {
            row_store<C, CS>(f0, xL + slot(yy + 1));
            row_store<C, CS>(f1, xL + slot(yy + 2));
            __syncthreads();
            const int base[4] = {slot(yy - 1), slot(yy), slot(yy + 1), slot(yy + 2)};
            const int xx = x0 + px;
            // input gradient: the ReLU masks of this lane's outputs, read now
            // so that they arrive during the products (and before the rows
            // fetched below, since loads complete in order)
            uint2 mk[2][NT] = {};
            if (MODE == kInputGrad && xx < W) {
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    if (yy + h < yb)
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            mk[h][nt] = *reinterpret_cast<const uint2*>(
                                mask + ((long long)(bimg * H + yy + h) * W + xx) * NOUT + nt * 16 + 4 * grp);
            }
            // in flight during the next two passes (issued in every pass, so
            // that the waits stay counted; rows past the run read nothing new)
            row_fetch<C>(f0, xr, H, W, yy + 5, x0, yy + 4 < yb);
            row_fetch<C>(f1, xr, H, W, yy + 6, x0, yy + 4 < yb);
            v4f acc[2][NT];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[h][nt] = v4f{0.f, 0.f, 0.f, 0.f};
            if constexpr (C == 32) {
                conv_pass32<CS, NT, sgn, TR>(xL, base, px * CS + 8 * grp, bw, acc);
            } else {
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int rs = rsel[ch];
                    const int o0 = (rs == 0 ? base[0] : rs == 1 ? base[1] : base[2]) + cofs[ch] + px * CS;
                    const int o1 = (rs == 0 ? base[1] : rs == 1 ? base[2] : base[3]) + cofs[ch] + px * CS;
                    const bf8 a0 = tap_ok[ch] ? __builtin_bit_cast(bf8, *reinterpret_cast<const v4u*>(xL + o0)) : zero8();
                    const bf8 a1 = tap_ok[ch] ? __builtin_bit_cast(bf8, *reinterpret_cast<const v4u*>(xL + o1)) : zero8();
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        if (TR) {
                            acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[ch][nt], a0, acc[0][nt], 0, 0, 0);
                            acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[ch][nt], a1, acc[1][nt], 0, 0, 0);
                        } else {
                            acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bw[ch][nt], acc[0][nt], 0, 0, 0);
                            acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bw[ch][nt], acc[1][nt], 0, 0, 0);
                        }
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int yo = yy + h;
                if (yo >= yb) break;
                const long long rowp = (long long)(bimg * H + yo) * W;
                if (MODE == kLast) {
                    // lane holds D[4 grp + r][i]: pixel 16 wv + 4 grp + r, output channel i (z is channel 0)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int xz = x0 + 16 * wv + 4 * grp + r;
                        if (xz < W && i == 0) z[rowp + xz] = acc[h][0][r];
                    }
                } else if (xx < W) {
                    // lane holds D[4 grp + r][i]: output channels nt*16 + 4 grp + r of pixel px
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        uint2 v = pack4(acc[h][nt], MODE == kHidden);
                        // input gradient: kept where the layer input (post-ReLU) is positive
                        if (MODE == kInputGrad) v = relu_mask(v, mk[h][nt]);
                        *reinterpret_cast<uint2*>(y + (rowp + xx) * NOUT + nt * 16 + 4 * grp) = v;
                    }
                }
            }
        };
        for (int yy = ya; yy < yb; yy += 4) {
            pass(yy, fa0, fa1);
            if (yy + 2 >= yb) break;
            pass(yy + 2, fc0, fc1);
        }
    }
}

// Weight gradient: part[block][tap][co][ci] = sum over the block's pixels p of
// dy[p][co] x[p + off(tap)][ci] (FP32 partials, summed over blocks in a fixed
// order by the reduction below).  A block of three waves owns a 32-pixel
// column segment of one image over a run of rows and walks down it: an LDS
// ring of four row slots holds input rows y-1 .. y+1 (columns x0-1 .. x0+32,
// zeros outside the image), dy of row y sits beside it, and the next rows of
// x and dy are fetched into registers while the current row runs on the
// matrix cores.
// Wave r accumulates the three taps of tap row r as GEMMs over the row's
// pixels on v_mfma_f32_16x16x32_bf16: A = dy^T (co x pixels), B = x shifted
// by the tap (pixels x ci).  A fragment takes 8 consecutive pixels of one
// channel: the LDS pixel stride is padded by two channels so that those
// gathers do not collide in the LDS banks.  The x ring has four slots and dy
// two, so the rows being written are never the ones being read and one
// barrier per row orders the two.  Blocks take (image, row run, segment)
// items with a grid stride and keep accumulating across them.
constexpr int kSeg = 32;
constexpr int kWgradMaxBlocks = 1024;
constexpr int kWgradRows = 16;

template <int C>
__device__ __forceinline__ bf8 gather8(const bf16* base) {  // base[s * (C + 2)], s = 0..7
    v4u v;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        v[k] = (unsigned)base[(2 * k) * (C + 2)] | ((unsigned)base[(2 * k + 1) * (C + 2)] << 16);
    return __builtin_bit_cast(bf8, v);
}

// One staged row of NPX pixels x C channels as 16-byte pieces, one per thread
// of the 192-thread block (NPX * C / 8 <= 192).
template <int C, int NPX>
struct WRow {
    static_assert(NPX * (C / 8) <= 192, "one piece per thread");
    v4u v;
};

template <int C, int NPX>
__device__ __forceinline__ void wrow_fetch(WRow<C, NPX>& f, const bf16* __restrict__ src, int bimg, int H, int W,
                                           int yy, int xs) {
    const int e = threadIdx.x;
    const int cg = e % (C / 8), j = e / (C / 8);
    const int xx = xs + j;
    v4u v = v4u{0u, 0u, 0u, 0u};
    if (e < NPX * (C / 8) && yy >= 0 && yy < H && xx >= 0 && xx < W)
        v = *reinterpret_cast<const v4u*>(src + ((long long)(bimg * H + yy) * W + xx) * C + cg * 8);
    f.v = v;
}

template <int C, int NPX>
__device__ __forceinline__ void wrow_store(const WRow<C, NPX>& f, bf16* row) {
    const int e = threadIdx.x;
    const int cg = e % (C / 8), j = e / (C / 8);
    if (e < NPX * (C / 8)) {
        unsigned* dst = reinterpret_cast<unsigned*>(row + j * (C + 2) + cg * 8);
#pragma unroll
        for (int k = 0; k < 4; ++k) dst[k] = f.v[k];
    }
}

template <int CIN, int COUT>
__global__ __launch_bounds__(192) void k_conv_wgrad(int B, int H, int W, const bf16* __restrict__ dy,
                                                   const bf16* __restrict__ x, float* __restrict__ part) {
    constexpr int XR = (kSeg + 2) * (CIN + 2);  // one staged x row
    constexpr int DR = kSeg * (COUT + 2);        // one staged dy row
    __shared__ bf16 dyL[2 * DR];
    __shared__ bf16 xL[4 * XR];
    constexpr int MT = COUT / 16, NT = CIN / 16;
    const int lane = threadIdx.x & 63, r = threadIdx.x >> 6;  // r: tap row (dy offset r - 1)
    const int i = lane & 15, grp = lane >> 4;
    const int segs_x = (W + kSeg - 1) / kSeg;
    const int runs = (H + kWgradRows - 1) / kWgradRows;
    const int nwork = B * runs * segs_x;
    v4f acc[3][MT][NT];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b) acc[d][a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int wk = blockIdx.x; wk < nwork; wk += gridDim.x) {
        const int sx = wk % segs_x, t = wk / segs_x;
        const int run = t % runs, bimg = t / runs;
        const int x0 = sx * kSeg, ya = run * kWgradRows, yb = min(H, ya + kWgradRows);
        WRow<CIN, kSeg + 2> fx;
        WRow<COUT, kSeg> fd;
        __syncthreads();  // the previous item's LDS reads are done
        wrow_fetch(fx, x, bimg, H, W, ya - 1, x0 - 1);
        wrow_store(fx, xL + ((ya + 3) & 3) * XR);
        wrow_fetch(fx, x, bimg, H, W, ya, x0 - 1);
        wrow_store(fx, xL + (ya & 3) * XR);
        wrow_fetch(fx, x, bimg, H, W, ya + 1, x0 - 1);
        wrow_fetch(fd, dy, bimg, H, W, ya, x0);
        for (int yy = ya; yy < yb; ++yy) {
            // x row yy+1 into the slot of row yy-3, dy row yy into the slot of row yy-2
            wrow_store(fx, xL + ((yy + 1) & 3) * XR);
            bf16* dyr = dyL + (yy & 1) * DR;
            wrow_store(fd, dyr);
            __syncthreads();
            if (yy + 1 < yb) {  // in flight during the products
                wrow_fetch(fx, x, bimg, H, W, yy + 2, x0 - 1);
                wrow_fetch(fd, dy, bimg, H, W, yy + 1, x0);
            }
            // K = the row's 32 pixels, one 32-deep MFMA step per tile
            bf8 A[MT];
#pragma unroll
            for (int a = 0; a < MT; ++a) A[a] = gather8<COUT>(dyr + (8 * grp) * (COUT + 2) + a * 16 + i);
            const bf16* xr = xL + ((yy + r + 3) & 3) * XR;  // x row yy + r - 1
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int b = 0; b < NT; ++b) {
                    const bf8 Bf = gather8<CIN>(xr + (8 * grp + d) * (CIN + 2) + b * 16 + i);
#pragma unroll
                    for (int a = 0; a < MT; ++a)
                        acc[d][a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a], Bf, acc[d][a][b], 0, 0, 0);
                }
            }
        }
    }
    // lane holds D[4 grp + q][i]: co = a*16 + 4 grp + q, ci = b*16 + i; tap = 3 r + d
    float* out = part + (long long)blockIdx.x * 9 * COUT * CIN;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    out[((3 * r + d) * COUT + a * 16 + 4 * grp + q) * CIN + b * 16 + i] = acc[d][a][b][q];
}

// Chunk partials -> weight gradient in two fixed-order FP64 stages: group g
// of kRedGroups sums its contiguous run of chunks (coalesced over the
// partial layout [chunk][tap][co][ci]), then the groups are summed in order
// into grad[co][ci][tap] (real channels only).
constexpr int kRedGroups = 32;

__global__ void k_wgrad_reduce1(int nchunk, int m, const float* __restrict__ part, double* __restrict__ gsum) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int gidx = blockIdx.y;
    if (e >= m) return;
    const int c0 = (int)((long long)nchunk * gidx / kRedGroups), c1 = (int)((long long)nchunk * (gidx + 1) / kRedGroups);
    double acc = 0.0;
    for (int c = c0; c < c1; ++c) acc += part[(long long)c * m + e];
    gsum[(long long)gidx * m + e] = acc;
}

__global__ void k_wgrad_reduce2(int m, int coutp, int cinp, int cout, int cin, const double* __restrict__ gsum,
                                float* __restrict__ grad) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= cout * cin * 9) return;
    const int tap = idx % 9, ci = (idx / 9) % cin, co = idx / (9 * cin);
    const int e = (tap * coutp + co) * cinp + ci;
    double acc = 0.0;
    for (int gidx = 0; gidx < kRedGroups; ++gidx) acc += gsum[(long long)gidx * m + e];
    grad[idx] = (float)acc;
}

// ---------------------------------------------------------------------------
// per-image FP64 reductions (fixed order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int NV>
__device__ __forceinline__ void block_store(double (&v)[NV], double* dst) {
    __shared__ double sh[4][NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = wave_sum(v[k]);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) dst[threadIdx.x] = sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
}

// image b, block k: partial sums of g^2, m, m^2
__global__ __launch_bounds__(256) void k_input_stats(int n, const float* __restrict__ g, const float* __restrict__ m,
                                                     double* __restrict__ part) {
    const int b = blockIdx.y;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += kRedBlocks * 256) {
        const double gv = g[(long long)b * n + i], mv = m[(long long)b * n + i];
        v[0] += gv * gv;
        v[1] += mv;
        v[2] += mv * mv;
    }
    block_store<3>(v, part + ((long long)b * kRedBlocks + blockIdx.x) * 3);
}

template <int NV>
__global__ void k_finish(int B, const double* __restrict__ part, double* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    for (int k = 0; k < NV; ++k) {
        double acc = 0.0;
        for (int j = 0; j < kRedBlocks; ++j) acc += part[((long long)b * kRedBlocks + j) * NV + k];
        out[b * NV + k] = acc;
    }
}

// a0[p][0] = g / rms(g), a0[p][1] = (m - mean) / std, channels 2..15 zero
__global__ void k_pack_input(int B, int n, const float* __restrict__ g, const float* __restrict__ m,
                             const double* __restrict__ st, bf16* __restrict__ a0) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (long long)B * n) return;
    const int b = (int)(p / n);
    const double rg = sqrt(st[b * 3] / n);
    const double mean = st[b * 3 + 1] / n;
    const double var = fmax(st[b * 3 + 2] / n - mean * mean, 0.0);
    const double sd = sqrt(var);
    const float gh = rg > 0 ? (float)(g[p] / rg) : 0.f;
    const float mh = sd > 0 ? (float)((m[p] - mean) / sd) : 0.f;
    bf16* o = a0 + p * 16;
    o[0] = f2bf(gh);
    o[1] = f2bf(mh);
#pragma unroll
    for (int c = 2; c < 16; ++c) o[c] = 0;
}

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoidf(float z) { return 1.f / (1.f + expf(-z)); }

// d = softplus(z) * g
__global__ void k_direction(long long N, const float* __restrict__ z, const float* __restrict__ g, float* __restrict__ d) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) d[i] = softplusf(z[i]) * g[i];
}

// pass 1 of the loss: sum d^2 and sum s^2 per image
__global__ __launch_bounds__(256) void k_loss_a(int n, const float* __restrict__ z, const float* __restrict__ g,
                                                const float* __restrict__ s, double* __restrict__ part) {
    const int b = blockIdx.y;
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += kRedBlocks * 256) {
        const long long o = (long long)b * n + i;
        const double d = (double)softplusf(z[o]) * g[o];
        v[0] += d * d;
        v[1] += (double)s[o] * s[o];
    }
    block_store<2>(v, part + ((long long)b * kRedBlocks + blockIdx.x) * 2);
}

// pass 2: sum (u - t) u and sum (u - t)^2 with u = d / rms(d), t = -s / rms(s)
__global__ __launch_bounds__(256) void k_loss_b(int n, const float* __restrict__ z, const float* __restrict__ g,
                                                const float* __restrict__ s, const double* __restrict__ st1,
                                                double* __restrict__ part) {
    const int b = blockIdx.y;
    const double rd = sqrt(st1[b * 2] / n), rs = sqrt(st1[b * 2 + 1] / n);
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += kRedBlocks * 256) {
        const long long o = (long long)b * n + i;
        const double u = (double)softplusf(z[o]) * g[o] / rd;
        const double e = u + (double)s[o] / rs;
        v[0] += e * u;
        v[1] += e * e;
    }
    block_store<2>(v, part + ((long long)b * kRedBlocks + blockIdx.x) * 2);
}

// pass 3: dL/dz = (2/(n rd)) [e - u mean(e u)] g sigmoid(z) / B, packed as
// channel 0 of a 16-channel bf16 tensor
__global__ void k_loss_c(int B, int n, const float* __restrict__ z, const float* __restrict__ g,
                         const float* __restrict__ s, const double* __restrict__ st1, const double* __restrict__ st2,
                         bf16* __restrict__ dz16) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (long long)B * n) return;
    const int b = (int)(p / n);
    const double rd = sqrt(st1[b * 2] / n), rs = sqrt(st1[b * 2 + 1] / n);
    const double u = (double)softplusf(z[p]) * g[p] / rd;
    const double e = u + (double)s[p] / rs;
    const double dd = 2.0 / (n * rd) * (e - u * st2[b * 2] / n);
    const float dzv = (float)(dd * g[p] * sigmoidf(z[p]) / B);
    bf16* o = dz16 + p * 16;
    o[0] = f2bf(dzv);
#pragma unroll
    for (int c = 1; c < 16; ++c) o[c] = 0;
}

__global__ void k_loss_total(int B, int n, const double* __restrict__ st2, double* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double acc = 0.0;
    for (int b = 0; b < B; ++b) acc += st2[b * 2 + 1] / n;
    loss[0] = acc / B;
}

// Adam on FP32 master weights.
__global__ void k_adam(int n, float lr, float b1, float b2, float eps, float c1, float c2, float* __restrict__ w,
                       float* __restrict__ mo, float* __restrict__ vo, const float* __restrict__ gr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float m = b1 * mo[i] + (1.f - b1) * g;
    const float v = b2 * vo[i] + (1.f - b2) * g * g;
    mo[i] = m;
    vo[i] = v;
    w[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Layers 2 and 3 in one pass (32 -> 32 -> 32, ReLU after each): layer 3's
// input, h2 = ReLU(conv(h1, W2)), is computed into an LDS ring of rows and
// consumed there, so it never goes to HBM unless the caller keeps it (the
// training forward keeps it for the backward pass).  A block of four waves
// owns layer 3's outputs on kFSeg = 62 columns [x0, x0+62) of one image over
// a run of rows; it evaluates h2 on the 64 columns [x0-1, x0+63) (one
// 16-pixel MFMA tile per wave) from h1 on [x0-2, x0+64), and h2 is set to
// zero outside the image, which is the zero padding layer 3 sees when h2
// comes from HBM.  Per pass, h2 rows yy+1 and yy+2 are added to the h2 ring
// (6 slots) from h1 rows yy .. yy+3 (6-slot ring, the next two fetched into
// registers during the products), then layer 3's rows yy and yy+1 are
// produced from h2 rows yy-1 .. yy+2.  Both layers' weight fragments stay in
// registers.  Every product runs in the order of the single-layer kernel on
// the same bf16 values, so the outputs are bitwise those of two separate
// layers.
constexpr int kFSeg = 62;

template <bool KEEP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_fused23(int B, int H, int W, int rows, const bf16* __restrict__ x,
                                                      const bf16* __restrict__ w2, const bf16* __restrict__ w3,
                                                      bf16* __restrict__ h2out, bf16* __restrict__ y) {
    constexpr int C = 32, NOUT = 32, NT = NOUT / 16;
    constexpr int CS = C + 8;             // LDS pixel stride of both rings
    constexpr int RW = (kCSeg + 2) * CS;  // h1 row: columns x0-2 .. x0+63; h2 row: x0-1 .. x0+62, two zero pixels after
    __shared__ __align__(16) bf16 xL[kConvSlots * RW];
    __shared__ __align__(16) bf16 hL[kConvSlots * RW];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = lane & 15, grp = lane >> 4;
    bf8 bw2[9][NT], bw3[9][NT];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            bw2[t][nt] = ld8(w2 + ((t * NOUT + nt * 16 + i) * C + 8 * grp));
            bw3[t][nt] = ld8(w3 + ((t * NOUT + nt * 16 + i) * C + 8 * grp));
        }
    settle(bw2);
    settle(bw3);
    // the two pixels after the 64 h2 columns are read (and discarded) by
    // layer 3's last two output pixels: keep them zero in every slot
    for (int e = threadIdx.x; e < kConvSlots * 2 * CS; e += 256) {
        const int sl = e / (2 * CS), r = e % (2 * CS);
        hL[sl * RW + kCSeg * CS + r] = (bf16)0;
    }
    auto slot = [](int r) { return ((r + 2 * kConvSlots) % kConvSlots) * RW; };  // r >= -2
    const int segs_x = (W + kFSeg - 1) / kFSeg;
    const int runs = (H + rows - 1) / rows;
    const int nwork = B * runs * segs_x;
    const int px = 16 * wv + i;  // this lane's pixel (B columns) in both layers' 64-pixel tiles
    const int aofs = px * CS + 8 * grp;
    for (int wk = blockIdx.x; wk < nwork; wk += gridDim.x) {
        const int sx = wk % segs_x, t = wk / segs_x;
        const int run = t % runs, bimg = t / runs;
        const int x0 = sx * kFSeg, ya = run * rows, yb = min(H, ya + rows);
        // layer 2 on h2 rows r, r+1 (h1 rows r-1 .. r+2 in the ring): ReLU,
        // zero outside the image, bf16 into the h2 ring (and, when kept, the
        // rows and columns this block owns to HBM)
        auto layer2 = [&](int r) {
            const int base[4] = {slot(r - 1), slot(r), slot(r + 1), slot(r + 2)};
            v4f acc[2][NT];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[h][nt] = v4f{0.f, 0.f, 0.f, 0.f};
            conv_pass32<CS, NT, 1, true>(xL, base, aofs, bw2, acc);
            const int xx = x0 - 1 + px;  // h2 pixel px is column x0 - 1 + px
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int yo = r + h;
                const bool in = yo >= 0 && yo < H && xx >= 0 && xx < W;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const uint2 v = in ? pack4(acc[h][nt], true) : uint2{0u, 0u};
                    *reinterpret_cast<uint2*>(hL + slot(yo) + px * CS + nt * 16 + 4 * grp) = v;
                    if (KEEP && in && yo >= ya && yo < yb && px >= 1 && px <= kFSeg)
                        *reinterpret_cast<uint2*>(h2out + ((long long)(bimg * H + yo) * W + xx) * C + nt * 16 + 4 * grp) = v;
                }
            }
        };
        // h1 rows of the next two passes are in flight in registers (two
        // buffer pairs, alternating between passes)
        const Rsrc xr = image_view<C>(x, bimg, H, W);
        RowFetch<C> fa0, fa1, fc0, fc1;
        __syncthreads();  // the rings' previous contents are no longer read
        // h1 rows ya-2 .. ya+1 (columns x0-2 .. x0+63) for h2 rows ya-1, ya
        row_fetch<C>(fa0, xr, H, W, ya - 2, x0 - 1);
        row_fetch<C>(fa1, xr, H, W, ya - 1, x0 - 1);
        row_fetch<C>(fc0, xr, H, W, ya, x0 - 1);
        row_fetch<C>(fc1, xr, H, W, ya + 1, x0 - 1);
        row_store<C, CS>(fa0, xL + slot(ya - 2));
        row_store<C, CS>(fa1, xL + slot(ya - 1));
        row_store<C, CS>(fc0, xL + slot(ya));
        row_store<C, CS>(fc1, xL + slot(ya + 1));
        row_fetch<C>(fa0, xr, H, W, ya + 2, x0 - 1);
        row_fetch<C>(fa1, xr, H, W, ya + 3, x0 - 1);
        row_fetch<C>(fc0, xr, H, W, ya + 4, x0 - 1, ya + 2 < yb);
        row_fetch<C>(fc1, xr, H, W, ya + 5, x0 - 1, ya + 2 < yb);
        __syncthreads();
        layer2(ya - 1);
        auto pass = [&](int yy, RowFetch<C>& f0, RowFetch<C>& f1) {
            // h1 rows yy+2, yy+3 go to the slots of rows yy-4, yy-3
            row_store<C, CS>(f0, xL + slot(yy + 2));
            row_store<C, CS>(f1, xL + slot(yy + 3));
            __syncthreads();
            // rows of the pass after next (issued in every pass, so that the
            // waits stay counted; rows past the run read nothing new)
            row_fetch<C>(f0, xr, H, W, yy + 6, x0 - 1, yy + 4 < yb);
            row_fetch<C>(f1, xr, H, W, yy + 7, x0 - 1, yy + 4 < yb);
            layer2(yy + 1);  // h2 rows yy+1, yy+2 into the slots of rows yy-5, yy-4
            __syncthreads();
            const int base[4] = {slot(yy - 1), slot(yy), slot(yy + 1), slot(yy + 2)};
            v4f acc[2][NT];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[h][nt] = v4f{0.f, 0.f, 0.f, 0.f};
            conv_pass32<CS, NT, 1, true>(hL, base, aofs, bw3, acc);
            const int xx = x0 + px;  // output pixel px is column x0 + px
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int yo = yy + h;
                if (yo >= yb) break;
                if (px < kFSeg && xx < W) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        *reinterpret_cast<uint2*>(y + ((long long)(bimg * H + yo) * W + xx) * NOUT + nt * 16 + 4 * grp) =
                            pack4(acc[h][nt], true);
                }
            }
        };
        for (int yy = ya; yy < yb; yy += 4) {
            pass(yy, fa0, fa1);
            if (yy + 2 >= yb) break;
            pass(yy + 2, fc0, fc1);
        }
    }
}

// bf16 copies: Wf[tap][co][ci] and Wd[tap][ci][co] (padded with zeros)
__global__ void k_pack_weights(int cout, int cin, int coutp, int cinp, const float* __restrict__ w,
                               bf16* __restrict__ wf, bf16* __restrict__ wd) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 9 * coutp * cinp) return;
    const int ci = idx % cinp, co = (idx / cinp) % coutp, tap = idx / (cinp * coutp);
    const float v = (co < cout && ci < cin) ? w[(co * cin + ci) * 9 + tap] : 0.f;
    const bf16 h = f2bf(v);
    wf[(tap * coutp + co) * cinp + ci] = h;
    if (wd) wd[(tap * cinp + ci) * coutp + co] = h;
}

}  // namespace
}  // namespace aafwi

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using aafwi::Error;

struct aafwi_cnn {
    int H = 0, W = 0, Bmax = 0;
    hipStream_t stream = nullptr;
    int step = 0;
    std::vector<void*> allocs;
    float* w = nullptr;     // FP32 master weights (AAFWI_CNN_PARAMS)
    float* mo = nullptr;    // Adam moments
    float* vo = nullptr;
    float* grad = nullptr;
    aafwi::bf16* wf[aafwi::kL] = {};
    aafwi::bf16* wd[aafwi::kL] = {};
    aafwi::bf16* act[aafwi::kL] = {};  // inputs of layers 1..4 (a0..a3)
    aafwi::bf16* dlt[aafwi::kL] = {};  // deltas at the outputs of layers 1..4
    float* z = nullptr;
    double* part = nullptr;
    double* st_in = nullptr;
    double* st1 = nullptr;
    double* st2 = nullptr;
    float* wpart = nullptr;
    double* gsum = nullptr;
    bool fused = true;  // layers 2 and 3 in one kernel (bitwise the same outputs)
};

namespace {

template <typename F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        aafwi::set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        aafwi::set_last_error("host allocation failed");
        return AAFWI_E_NOMEM;
    } catch (...) {
        aafwi::set_last_error("unknown error");
        return AAFWI_E_INVALID;
    }
}

template <typename T>
T* calloc_dev(aafwi_cnn* c, size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(T) * (n ? n : 1)) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{AAFWI_E_NOMEM, "cnn: device allocation failed"};
    }
    c->allocs.push_back(p);
    AAFWI_HIP(hipMemset(p, 0, sizeof(T) * (n ? n : 1)));
    return (T*)p;
}

int layer_offset(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += aafwi::kCout[i] * aafwi::kCin[i] * 9;
    return o;
}

void pack_weights(aafwi_cnn* c) {
    for (int l = 0; l < aafwi::kL; ++l) {
        const int n = 9 * aafwi::kCoutP[l] * aafwi::kCinP[l];
        hipLaunchKernelGGL(aafwi::k_pack_weights, dim3((n + 255) / 256), dim3(256), 0, c->stream, aafwi::kCout[l],
                           aafwi::kCin[l], aafwi::kCoutP[l], aafwi::kCinP[l], c->w + layer_offset(l), c->wf[l], c->wd[l]);
        AAFWI_HIP(hipGetLastError());
    }
}

template <int C, int NOUT, int MODE>
void conv(aafwi_cnn* c, int B, const aafwi::bf16* x, const aafwi::bf16* w, const aafwi::bf16* mask, aafwi::bf16* y,
          float* z) {
    // runs of 16 rows, shorter when that leaves fewer than ~2 blocks per CU
    const int segs = B * ((c->W + aafwi::kCSeg - 1) / aafwi::kCSeg);
    int rows = 16;
    while (rows > 4 && segs * ((c->H + rows - 1) / rows) < 512) rows /= 2;
    const int nwork = segs * ((c->H + rows - 1) / rows);
    const int blocks = std::min(nwork, 2048);
    hipLaunchKernelGGL((aafwi::k_conv_mm<C, NOUT, MODE>), dim3(blocks), dim3(256), 0, c->stream, B, c->H, c->W, rows,
                       x, w, mask, y, z);
}

void weight_reduce(aafwi_cnn* c, int nchunk, int coutp, int cinp, int layer) {
    using namespace aafwi;
    const int m = 9 * coutp * cinp;
    hipLaunchKernelGGL(k_wgrad_reduce1, dim3((m + 255) / 256, kRedGroups), dim3(256), 0, c->stream, nchunk, m,
                       (const float*)c->wpart, c->gsum);
    hipLaunchKernelGGL(k_wgrad_reduce2, dim3((kCout[layer] * kCin[layer] * 9 + 255) / 256), dim3(256), 0, c->stream,
                       m, coutp, cinp, kCout[layer], kCin[layer], (const double*)c->gsum, c->grad + layer_offset(layer));
}

// Layers 2 and 3 fused (h2 kept in HBM only when the backward pass needs it).
void conv_fused23(aafwi_cnn* c, int B, bool keep) {
    const int segs = B * ((c->W + aafwi::kFSeg - 1) / aafwi::kFSeg);
    int rows = 16;
    while (rows > 4 && segs * ((c->H + rows - 1) / rows) < 512) rows /= 2;
    const int nwork = segs * ((c->H + rows - 1) / rows);
    const int blocks = std::min(nwork, 2048);
    if (keep)
        hipLaunchKernelGGL((aafwi::k_conv_fused23<true>), dim3(blocks), dim3(256), 0, c->stream, B, c->H, c->W, rows,
                           c->act[1], c->wf[1], c->wf[2], c->act[2], c->act[3]);
    else
        hipLaunchKernelGGL((aafwi::k_conv_fused23<false>), dim3(blocks), dim3(256), 0, c->stream, B, c->H, c->W, rows,
                           c->act[1], c->wf[1], c->wf[2], nullptr, c->act[3]);
}

void forward(aafwi_cnn* c, int B, const float* g, const float* m, bool keep = true) {
    using namespace aafwi;
    const int n = c->H * c->W, P = B * n;
    hipLaunchKernelGGL(k_input_stats, dim3(kRedBlocks, B), dim3(256), 0, c->stream, n, g, m, c->part);
    hipLaunchKernelGGL(k_finish<3>, dim3((B + 63) / 64), dim3(64), 0, c->stream, B, (const double*)c->part, c->st_in);
    hipLaunchKernelGGL(k_pack_input, dim3((P + 255) / 256), dim3(256), 0, c->stream, B, n, g, m,
                       (const double*)c->st_in, c->act[0]);
    conv<16, 32, kHidden>(c, B, c->act[0], c->wf[0], nullptr, c->act[1], nullptr);
    if (c->fused) {
        conv_fused23(c, B, keep);
    } else {
        conv<32, 32, kHidden>(c, B, c->act[1], c->wf[1], nullptr, c->act[2], nullptr);
        conv<32, 32, kHidden>(c, B, c->act[2], c->wf[2], nullptr, c->act[3], nullptr);
    }
    conv<32, 16, kLast>(c, B, c->act[3], c->wf[3], nullptr, nullptr, c->z);
    AAFWI_HIP(hipGetLastError());
}

// forward, loss and weight gradient (into c->grad); loss (device double) optional
void gradients(aafwi_cnn* c, int B, const float* g, const float* m, const float* s, double* loss) {
    using namespace aafwi;
    forward(c, B, g, m);
    const int n = c->H * c->W, P = B * n;
    hipLaunchKernelGGL(k_loss_a, dim3(kRedBlocks, B), dim3(256), 0, c->stream, n, (const float*)c->z, g, s, c->part);
    hipLaunchKernelGGL(k_finish<2>, dim3((B + 63) / 64), dim3(64), 0, c->stream, B, (const double*)c->part, c->st1);
    hipLaunchKernelGGL(k_loss_b, dim3(kRedBlocks, B), dim3(256), 0, c->stream, n, (const float*)c->z, g, s,
                       (const double*)c->st1, c->part);
    hipLaunchKernelGGL(k_finish<2>, dim3((B + 63) / 64), dim3(64), 0, c->stream, B, (const double*)c->part, c->st2);
    hipLaunchKernelGGL(k_loss_c, dim3((P + 255) / 256), dim3(256), 0, c->stream, B, n, (const float*)c->z, g, s,
                       (const double*)c->st1, (const double*)c->st2, c->dlt[3]);
    if (loss) hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, c->stream, B, n, (const double*)c->st2, loss);
    AAFWI_HIP(hipGetLastError());
    const int nwork = B * ((c->H + kWgradRows - 1) / kWgradRows) * ((c->W + kSeg - 1) / kSeg);
    const int nchunk = std::min(nwork, kWgradMaxBlocks);
    // layer 4 (32 -> 1): weight gradient, then the delta at layer 3's output
    hipLaunchKernelGGL((k_conv_wgrad<32, 16>), dim3(nchunk), dim3(192), 0, c->stream, B, c->H, c->W, c->dlt[3],
                       c->act[3], c->wpart);
    weight_reduce(c, nchunk, 16, 32, 3);
    conv<16, 32, kInputGrad>(c, B, c->dlt[3], c->wd[3], c->act[3], c->dlt[2], nullptr);
    for (int l = 2; l >= 1; --l) {
        hipLaunchKernelGGL((k_conv_wgrad<32, 32>), dim3(nchunk), dim3(192), 0, c->stream, B, c->H, c->W, c->dlt[l],
                           c->act[l], c->wpart);
        weight_reduce(c, nchunk, 32, 32, l);
        conv<32, 32, kInputGrad>(c, B, c->dlt[l], c->wd[l], c->act[l], c->dlt[l - 1], nullptr);
    }
    hipLaunchKernelGGL((k_conv_wgrad<16, 32>), dim3(nchunk), dim3(192), 0, c->stream, B, c->H, c->W, c->dlt[0],
                       c->act[0], c->wpart);
    weight_reduce(c, nchunk, 32, 16, 0);
    AAFWI_HIP(hipGetLastError());
}

void check_batch(const aafwi_cnn* c, int B) {
    AAFWI_REQUIRE(B >= 1 && B <= c->Bmax, "cnn: batch size outside [1, max_batch]");
}

}  // namespace

extern "C" int aafwi_cnn_create(int32_t nz, int32_t nx, int32_t max_batch, const float* weights, aafwi_stream stream,
                                aafwi_cnn** out) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(out && weights, "cnn_create: NULL argument");
        AAFWI_REQUIRE(nz >= 1 && nx >= 1 && max_batch >= 1, "cnn_create: bad size");
        AAFWI_REQUIRE((long long)nz * nx * max_batch < (1LL << 31), "cnn_create: too many pixels");
        // one image's 32-channel bf16 activations are addressed with 32-bit byte offsets
        AAFWI_REQUIRE((long long)nz * nx * 64 < (1LL << 31), "cnn_create: an image of more than 2^25 pixels");
        *out = nullptr;
        aafwi_cnn* c = new aafwi_cnn{};
        try {
            c->H = nz;
            c->W = nx;
            c->Bmax = max_batch;
            c->stream = (hipStream_t)stream;
            const size_t P = (size_t)nz * nx * max_batch;
            c->w = calloc_dev<float>(c, AAFWI_CNN_PARAMS);
            c->mo = calloc_dev<float>(c, AAFWI_CNN_PARAMS);
            c->vo = calloc_dev<float>(c, AAFWI_CNN_PARAMS);
            c->grad = calloc_dev<float>(c, AAFWI_CNN_PARAMS);
            for (int l = 0; l < aafwi::kL; ++l) {
                c->wf[l] = calloc_dev<aafwi::bf16>(c, 9 * aafwi::kCoutP[l] * aafwi::kCinP[l]);
                c->wd[l] = calloc_dev<aafwi::bf16>(c, 9 * aafwi::kCoutP[l] * aafwi::kCinP[l]);
                c->act[l] = calloc_dev<aafwi::bf16>(c, P * aafwi::kCinP[l]);
                c->dlt[l] = calloc_dev<aafwi::bf16>(c, P * aafwi::kCoutP[l]);
            }
            c->z = calloc_dev<float>(c, P);
            c->part = calloc_dev<double>(c, (size_t)max_batch * aafwi::kRedBlocks * 3);
            c->st_in = calloc_dev<double>(c, (size_t)max_batch * 3);
            c->st1 = calloc_dev<double>(c, (size_t)max_batch * 2);
            c->st2 = calloc_dev<double>(c, (size_t)max_batch * 2);
            const size_t nwork = (size_t)max_batch * ((nz + aafwi::kWgradRows - 1) / aafwi::kWgradRows) *
                                 ((nx + aafwi::kSeg - 1) / aafwi::kSeg);
            const size_t nchunk = std::min(nwork, (size_t)aafwi::kWgradMaxBlocks);
            c->wpart = calloc_dev<float>(c, nchunk * 9 * 32 * 32);
            c->gsum = calloc_dev<double>(c, (size_t)aafwi::kRedGroups * 9 * 32 * 32);
            AAFWI_HIP(hipMemcpy(c->w, weights, sizeof(float) * AAFWI_CNN_PARAMS, hipMemcpyHostToDevice));
            pack_weights(c);
            AAFWI_HIP(hipStreamSynchronize(c->stream));
        } catch (...) {
            for (void* p : c->allocs) (void)hipFree(p);
            delete c;
            throw;
        }
        *out = c;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_cnn_destroy(aafwi_cnn* c) {
    return guarded([&]() -> int {
        if (!c) return AAFWI_OK;
        (void)hipStreamSynchronize(c->stream);
        for (void* p : c->allocs) (void)hipFree(p);
        delete c;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_cnn_set_weights(aafwi_cnn* c, const float* weights) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && weights, "cnn_set_weights: NULL argument");
        AAFWI_HIP(hipStreamSynchronize(c->stream));
        AAFWI_HIP(hipMemcpy(c->w, weights, sizeof(float) * AAFWI_CNN_PARAMS, hipMemcpyHostToDevice));
        AAFWI_HIP(hipMemset(c->mo, 0, sizeof(float) * AAFWI_CNN_PARAMS));
        AAFWI_HIP(hipMemset(c->vo, 0, sizeof(float) * AAFWI_CNN_PARAMS));
        c->step = 0;
        pack_weights(c);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_cnn_get_weights(aafwi_cnn* c, float* weights) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && weights, "cnn_get_weights: NULL argument");
        AAFWI_HIP(hipStreamSynchronize(c->stream));
        AAFWI_HIP(hipMemcpy(weights, c->w, sizeof(float) * AAFWI_CNN_PARAMS, hipMemcpyDeviceToHost));
        return AAFWI_OK;
    });
}

extern "C" int aafwi_cnn_forward(aafwi_cnn* c, int32_t B, const float* g, const float* m, float* z, float* d) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && g && m, "cnn_forward: NULL argument");
        check_batch(c, B);
        forward(c, B, g, m, /*keep=*/false);
        const long long N = (long long)B * c->H * c->W;
        if (z) AAFWI_HIP(hipMemcpyAsync(z, c->z, sizeof(float) * N, hipMemcpyDeviceToDevice, c->stream));
        if (d) {
            hipLaunchKernelGGL(aafwi::k_direction, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c->stream, N,
                               (const float*)c->z, g, d);
            AAFWI_HIP(hipGetLastError());
        }
        return AAFWI_OK;
    });
}

extern "C" int aafwi_cnn_set_fused(aafwi_cnn* c, int32_t on) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c, "cnn_set_fused: NULL handle");
        c->fused = on != 0;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_cnn_gradients(aafwi_cnn* c, int32_t B, const float* g, const float* m, const float* s,
                                   float* grad, double* loss) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && g && m && s && grad, "cnn_gradients: NULL argument");
        check_batch(c, B);
        gradients(c, B, g, m, s, loss);
        AAFWI_HIP(hipMemcpyAsync(grad, c->grad, sizeof(float) * AAFWI_CNN_PARAMS, hipMemcpyDeviceToDevice, c->stream));
        return AAFWI_OK;
    });
}

extern "C" int aafwi_cnn_train_step(aafwi_cnn* c, int32_t B, const float* g, const float* m, const float* s, float lr,
                                    double* loss) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && g && m && s, "cnn_train_step: NULL argument");
        AAFWI_REQUIRE(std::isfinite(lr) && lr > 0, "cnn_train_step: lr must be positive");
        check_batch(c, B);
        gradients(c, B, g, m, s, loss);
        c->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - std::pow(b1, (float)c->step), c2 = 1.f - std::pow(b2, (float)c->step);
        hipLaunchKernelGGL(aafwi::k_adam, dim3((AAFWI_CNN_PARAMS + 255) / 256), dim3(256), 0, c->stream,
                           AAFWI_CNN_PARAMS, lr, b1, b2, 1e-8f, c1, c2, c->w, c->mo, c->vo, (const float*)c->grad);
        AAFWI_HIP(hipGetLastError());
        pack_weights(c);
        return AAFWI_OK;
    });
}
