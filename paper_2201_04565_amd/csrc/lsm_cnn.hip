// lsm_cnn.hip -- surrogate network of the lattice spring model (gfx950).
//
// A small CNN maps a two-phase image to the stress-strain curve and modulus
// that the batched lattice spring model produces for it (the paper motivates
// the code by data generation for machine-learning materials design,
// Abstract and Section 4).  Layers: five 3x3 convolutions (ReLU; 2x2 average
// pooling after the first four), global average pooling, two dense layers.
//
// Convolutions with at least 32 input channels are implicit GEMMs on the
// BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation): rows =
// output pixels, columns = output channels, reduction = 3x3 taps x input
// channels.  Activations are NHWC BF16, so both MFMA operands of the forward
// and input-gradient products are 16-byte vector loads; the weight gradient
// (reduction over pixels) stages transposed tiles in LDS and is split over
// pixel ranges with a fixed-order second pass (deterministic).  Master
// weights, Adam moments and dense layers are FP32.
//
// Pooling never makes a pass of its own: the first layer (one input
// channel) is computed and pooled by one kernel, which also keeps the ReLU
// signs for its backward pass; the other pooled layers pool in the conv
// epilogue and keep a 4-bit ReLU mask per pooled pixel, which the next
// layer's input-gradient epilogue uses to write the full-resolution gradient
// directly.  Only the last conv output is stored at full resolution.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lsm.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kLayers = 5;
constexpr int kBlk = 256;

__device__ inline u16 f2bf(float x) {
    // round to nearest even: one hardware conversion (v_cvt_pk_bf16_f32)
    return __builtin_bit_cast(u16, __bf16(x));
}
__device__ inline float bf2f(u16 h) { return __uint_as_float(unsigned(h) << 16); }

// Full-resolution gradient below a pooled layer from its pooled gradient
// g (BF16, eight channels) and the ReLU mask bytes of those channels: at
// sub-pixel d of a 2 x 2 quad, bf16(g / 4) where bit d is set, else 0 --
// the values the expanding epilogue stores.
__device__ inline uint4 expand8(uint4 g8, uint2 m8, int d) {
    const u16 *g = reinterpret_cast<const u16 *>(&g8);
    const uint8_t *m = reinterpret_cast<const uint8_t *>(&m8);
    u16 o[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = (m[e] >> d) & 1u ? f2bf(0.25f * bf2f(g[e])) : u16(0);
    return *reinterpret_cast<const uint4 *>(o);
}


union Frag {
    uint4 u;
    bf16x8 v;
};

// ------------------------------------------------------------------ conv 1
// First layer fused with its 2x2 pooling: one thread per pooled pixel, all
// C channels.  Each of the four conv outputs is rounded to BF16 after the
// ReLU and the four are averaged in the order (0,0), (0,1), (1,0), (1,1):
// the same values as storing the conv output and pooling it, without the
// full-resolution map ever reaching memory (its ReLU signs are kept, four
// bits per pooled pixel and channel).
__device__ inline void conv1_patch(const uint8_t *x, int H, int W, int64_t n, int yo, int xo, float v[4][4]) {
    // sixteen unconditional loads from clamped addresses, zeroed off the
    // image by a factor (a select would let the compiler put each load
    // behind a branch that waits for it)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int sy = 2 * yo - 1 + r;
        const int cy = min(max(sy, 0), H - 1);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int sx = 2 * xo - 1 + c;
            const int cx = min(max(sx, 0), W - 1);
            const float on = (sy >= 0 && sy < H && sx >= 0 && sx < W) ? 1.0f : 0.0f;
            v[r][c] = float(x[(n * H + cy) * W + cx]) * on;
        }
    }
}

// pooled pixel q -> (x, y, image); 32-bit division where q fits
__device__ inline void split_pooled(int64_t q, int Wo, int Ho, int &xo, int &yo, int64_t &n) {
    if (q <= 0x7FFFFFFF) {
        const uint32_t u = uint32_t(q), t = u / uint32_t(Wo);
        xo = int(u - t * uint32_t(Wo));
        yo = int(t % uint32_t(Ho));
        n = int64_t(t / uint32_t(Ho));
    } else {
        xo = int(q % Wo);
        yo = int((q / Wo) % Ho);
        n = q / (int64_t(Ho) * Wo);
    }
}

// conv output (before ReLU) of channel c at sub-pixel (dy, dx) of the patch
__device__ inline float conv1_at(const float *w, const float *b, int c, const float v[4][4], int dy, int dx) {
    float s = b[c];
#pragma unroll
    for (int t = 0; t < 9; ++t) s = fmaf(w[c * 9 + t], v[dy + t / 3][dx + t % 3], s);
    return s;
}

// The ReLU signs of the four conv outputs under each pooled pixel go to
// mask, 32 bits per group of eight channels (bit 4 e + d: channel 8 g + e,
// sub-pixel d = (d / 2, d mod 2)), for the backward pass.
__global__ __launch_bounds__(kBlk) void k_conv1_pool_fwd(const uint8_t *x, const float *w, const float *b,
                                                        u16 *pool, uint32_t *mask, int B, int H, int W, int C) {
    // weights and biases once per workgroup in LDS (C <= 256): every lane
    // reads the same word, a broadcast
    __shared__ float ws[256 * 9], bs[256];
    for (int t = threadIdx.x; t < C * 9; t += kBlk) ws[t] = w[t];
    for (int t = threadIdx.x; t < C; t += kBlk) bs[t] = b[t];
    __syncthreads();
    const int Ho = H / 2, Wo = W / 2;
    const int64_t q = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (q >= int64_t(B) * Ho * Wo) return;
    int xo, yo;
    int64_t n;
    split_pooled(q, Wo, Ho, xo, yo, n);
    float v[4][4];
    conv1_patch(x, H, W, n, yo, xo, v);
    // C is a multiple of 32: four groups of eight channels, one 16-byte mask store
    for (int c1 = 0; c1 < C; c1 += 32) {
        uint32_t mb[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
            const int c0 = c1 + 8 * gq;
            u16 h[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float s4 = 0.0f;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const float act = bf2f(f2bf(fmaxf(conv1_at(ws, bs, c0 + e, v, d >> 1, d & 1), 0.0f)));
                    mb[gq] |= act > 0.0f ? 1u << (4 * e + d) : 0u;
                    s4 += act;
                }
                h[e] = f2bf(0.25f * s4);
            }
            *reinterpret_cast<uint4 *>(pool + q * C + c0) = *reinterpret_cast<const uint4 *>(h);
        }
        *reinterpret_cast<uint4 *>(mask + q * (C / 8) + c1 / 8) = make_uint4(mb[0], mb[1], mb[2], mb[3]);
    }
}

// ------------------------------------------------------ implicit-GEMM conv
// out[p, co] = act(sum_{tap, ci} in[shift(p, tap), ci] * wt[co, tap, ci] + bias[co])
// in: [B, H, W, Cin] BF16, wt: [Cout, 9, Cin] BF16, out: [B, H, W, Cout] BF16.
// Each wavefront owns WM x WN MFMA tiles of 16 x 16 (WM * 16 pixels x WN *
// 16 channels); the four wavefronts of a workgroup stack along pixels.  The
// reduction runs in K steps of 32 (step kk covers tap kk / (Cin / 32),
// channels 32 (kk mod (Cin / 32)) onwards, i.e. weight columns 32 kk ..):
// a lane issues WM + WN 16-byte loads per step, one step ahead of the
// WM * WN MFMAs that consume them (two register stages).
template <int WM, int WN>
struct ConvOperands {
    Frag a[WM], b[WN];
};

template <int WM, int WN>
__device__ inline void conv_load_step(ConvOperands<WM, WN> &o, int kk, int ksteps_per_tap, const u16 *in,
                                      const int64_t *pbase, const int *py, const int *px, const bool *pok, int H,
                                      int W, int Cin, const u16 *const *wrow, const bool *cok, int kq) {
    const int tap = kk / ksteps_per_tap;
    const int ci0 = (kk - tap * ksteps_per_tap) * 32;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int64_t shift = (int64_t(dy) * W + dx) * Cin + ci0 + 8 * kq;
#pragma unroll
    for (int r = 0; r < WM; ++r) {
        const int sy = py[r] + dy, sx = px[r] + dx;
        const bool ok = pok[r] && sy >= 0 && sy < H && sx >= 0 && sx < W;
        const uint4 t = *reinterpret_cast<const uint4 *>(in + (ok ? pbase[r] + shift : 0));
        o.a[r].u = ok ? t : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < WN; ++c) {
        const uint4 t = *reinterpret_cast<const uint4 *>(wrow[c] + kk * 32);
        o.b[c].u = cok[c] ? t : make_uint4(0, 0, 0, 0);
    }
}

template <int WM, int WN>
__device__ inline void conv_mfma_step(f32x4 (&acc)[WM][WN], const ConvOperands<WM, WN> &o) {
#pragma unroll
    for (int r = 0; r < WM; ++r)
#pragma unroll
        for (int c = 0; c < WN; ++c)
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a[r].v, o.b[c].v, acc[r][c], 0, 0, 0);
}

// Epilogues of the implicit-GEMM convolution.
//  kEpiStore  out = bf16(relu(acc + bias)), one value per pixel
//  kEpiRaw    out = bf16(acc) (input gradient kept at its own resolution)
//  kEpiPool   forward conv followed by 2x2 average pooling: rows of a
//             16-row tile are four 2x2 quads (row m: quad m / 4, position
//             m mod 4 = (dy, dx) = (m / 2 mod 2, m mod 2)), so each lane holds
//             a whole quad of one channel; it stores the pooled value
//             bf16(0.25 (a0 + a1 + a2 + a3)) of the BF16 ReLU outputs a_i and
//             the 4-bit mask of a_i > 0 (one byte per pooled pixel and channel)
//  kEpiExpand input gradient of a layer whose input was pooled: the
//             gradient g = bf16(acc) of a pooled pixel becomes
//             bf16(0.25 g) on each of the four pixels below it whose ReLU
//             output was positive (mask from kEpiPool), 0 elsewhere
enum { kEpiStore = 0, kEpiRaw = 1, kEpiPool = 2, kEpiExpand = 3 };

template <int EPI, int WM, int WN>
__global__ __launch_bounds__(kBlk) void k_conv_mfma(const u16 *in, const u16 *wt, const float *bias, u16 *out,
                                                   const uint8_t *mask_in, uint8_t *mask_out, int B, int H, int W,
                                                   int Cin, int Cout) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t npix = int64_t(B) * H * W;
    const int64_t p0 = (int64_t(blockIdx.x) * 4 + wv) * (WM * 16);
    const int c0 = blockIdx.y * (WN * 16);
    const int r16 = lane & 15, kq = lane >> 4;  // row within the 16-tile, K quarter
    int py[WM], px[WM];
    int64_t pbase[WM];
    bool pok[WM];
#pragma unroll
    for (int r = 0; r < WM; ++r) {
        const int64_t p = p0 + r * 16 + r16;
        pok[r] = p < npix;
        const int64_t pp = pok[r] ? p : 0;
        if constexpr (EPI == kEpiPool) {
            // pp / 4 is a quad of the pooled grid, pp mod 4 its position
            const int Wq = W / 2, Hq = H / 2;
            const int64_t q = pp >> 2;
            const int sub = int(pp & 3);
            const int qx = int(q % Wq), qy = int((q / Wq) % Hq);
            const int64_t n = q / (int64_t(Hq) * Wq);
            px[r] = 2 * qx + (sub & 1);
            py[r] = 2 * qy + (sub >> 1);
            pbase[r] = ((n * H + py[r]) * W + px[r]) * Cin;
        } else {
            px[r] = int(pp % W);
            py[r] = int((pp / W) % H);
            pbase[r] = pp * Cin;
        }
    }
    f32x4 acc[WM][WN];
#pragma unroll
    for (int r = 0; r < WM; ++r)
#pragma unroll
        for (int c = 0; c < WN; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int K = 9 * Cin;
    const u16 *wrow[WN];
    bool cok[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) {
        const int co = c0 + c * 16 + r16;
        cok[c] = co < Cout;
        wrow[c] = wt + int64_t(cok[c] ? co : 0) * K + 8 * kq;
    }
    const int kpt = Cin / 32;
    const int nk = 9 * kpt;
    ConvOperands<WM, WN> s0, s1;
    conv_load_step<WM, WN>(s0, 0, kpt, in, pbase, py, px, pok, H, W, Cin, wrow, cok, kq);
    for (int kk = 0; kk < nk; kk += 2) {
        if (kk + 1 < nk) conv_load_step<WM, WN>(s1, kk + 1, kpt, in, pbase, py, px, pok, H, W, Cin, wrow, cok, kq);
        conv_mfma_step<WM, WN>(acc, s0);
        if (kk + 1 < nk) {
            if (kk + 2 < nk)
                conv_load_step<WM, WN>(s0, kk + 2, kpt, in, pbase, py, px, pok, H, W, Cin, wrow, cok, kq);
            conv_mfma_step<WM, WN>(acc, s1);
        }
    }
    // D layout: lane holds rows 4 * kq + i (pixels), column r16 (channel)
#pragma unroll
    for (int r = 0; r < WM; ++r)
#pragma unroll
        for (int c = 0; c < WN; ++c) {
            const int co = c0 + c * 16 + r16;
            if (co >= Cout) continue;
            if constexpr (EPI == kEpiPool) {
                const int64_t q = (p0 >> 2) + r * 4 + kq;  // this lane's quad
                if (4 * q >= npix) continue;
                const float bv = bias[co];
                float s4 = 0.0f;
                unsigned m = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float a = bf2f(f2bf(fmaxf(acc[r][c][i] + bv, 0.0f)));
                    s4 += a;
                    m |= (a > 0.0f ? 1u : 0u) << i;
                }
                out[q * Cout + co] = f2bf(0.25f * s4);
                mask_out[q * Cout + co] = uint8_t(m);
            } else if constexpr (EPI == kEpiExpand) {
                // output pixels are the pooled grid (H x W) of a 2H x 2W layer
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t p = p0 + r * 16 + 4 * kq + i;
                    if (p >= npix) continue;
                    const float g = 0.25f * bf2f(f2bf(acc[r][c][i]));
                    const u16 h = f2bf(g);
                    const unsigned m = mask_in[p * Cout + co];
                    const int x = int(p % W), y = int((p / W) % H);
                    const int64_t n = p / (int64_t(H) * W);
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const int64_t o = ((n * 2 * H + 2 * y + (d >> 1)) * (2 * W) + 2 * x + (d & 1)) * Cout + co;
                        out[o] = (m >> d) & 1u ? h : u16(0);
                    }
                }
            } else {
                const float bv = EPI == kEpiStore ? bias[co] : 0.0f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t p = p0 + r * 16 + 4 * kq + i;
                    if (p >= npix) continue;
                    float v = acc[r][c][i] + bv;
                    if (EPI == kEpiStore) v = fmaxf(v, 0.0f);
                    out[p * Cout + co] = f2bf(v);
                }
            }
        }
}

// Forward convolution (ReLU, then 2x2 average pooling or a plain store)
// with the input patch staged in LDS.  A workgroup computes an 8 x TW pixel
// tile of one image (TW = 8, 16 or 32) and BN output channels (32 to 128):
// the (8 + 2) x (TW + 2) x CIN input patch (zeros off the image) is loaded
// into LDS once and serves all nine taps, so each input value is fetched
// once per tile instead of once per tap.  A wavefront takes MT * 16 pixels
// (MT 16-row MFMA tiles of four 2x2 quads each, the row order of the
// pooling epilogue above) and the channels of its group: with 8 x 16 tiles
// and MT = 8 each of the four takes all 128 pixels and BN / 4 channels, with
// 8 x 32 tiles two take each half of the pixels for BN / 2 channels, with
// 8 x 8 tiles each takes all 64 pixels (MT = 4).  More pixels per wavefront
// means fewer weight loads per MFMA: on 8 x 16 tiles, 128-pixel wavefronts
// ran the layers 20-35 % faster than 64-pixel ones over BN / 2 channels,
// and 32-pixel ones over all BN channels 30-45 % slower.  The reduction runs in the same K steps and order as
// k_conv_mfma, so both kernels produce the same bits; weights come from
// global memory (L1/L2 resident), one step ahead.
// XIN: the input is the pooled gradient of the layer ([B][H/2][W/2][CIN])
// with the ReLU masks xmask of the layer below, expanded to H x W while the
// patch is staged (the full-resolution gradient is never stored).
template <int CIN, int TW, int BN, int EPI, int MT, bool XIN = false>
__device__ __attribute__((always_inline)) inline void conv_lds_body(const u16 *in, const u16 *wt, const float *bias,
                                                                    u16 *out, uint8_t *mask_out, int B, int H, int W,
                                                                    int Cout, const uint8_t *xmask = nullptr) {
    constexpr int PH = 10, PW = TW + 2;
    // u16 per staged pixel and per staged row: pixel strides of 4 (mod 32)
    // LDS banks and row strides of 16 put the eight pixels that one
    // 16-byte read phase touches (two quads) on distinct banks
    constexpr int PS = CIN + 8;
    constexpr int RS = PW * PS + 16;
    constexpr int KPT = CIN / 32;
    constexpr int NK = 9 * KPT;
    // MT 16-row MFMA tiles (MT * 16 pixels) x NT 16-column tiles per wavefront
    // the tile's 8 TW pixels form PG groups of MT * 16 (one per wavefront),
    // the BN channels CG groups: wavefront w takes pixel group w mod PG and
    // channel group w / PG
    constexpr int PG = 8 * TW / (16 * MT), CG = 4 / PG;
    static_assert(PG * 16 * MT == 8 * TW && PG * CG == 4 && BN % (16 * CG) == 0, "wavefront layout");
    constexpr int NT = BN / (16 * CG);
    constexpr int QW = TW / 2;            // quads per tile row pair
    __shared__ __attribute__((aligned(16))) u16 patch[PH * RS];
    const int tiles_x = W / TW, tiles_y = H / 8;
    const int tile = blockIdx.x;
    const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y;
    const int n = tile / (tiles_x * tiles_y);
    const int y0 = ty * 8, x0 = tx * TW;
    // patch copy: every round's loads (unconditional, from the image's first
    // pixel off the image, zeroed afterwards), then the stores, so no round
    // waits for the previous one's load
    {
        constexpr int NCH = PH * PW * (CIN / 8), NR = (NCH + kBlk - 1) / kBlk;
        uint4 v[NR];
        uint2 vm[XIN ? NR : 1];
#pragma unroll
        for (int it = 0; it < NR; ++it) {
            const int idx = min(int(threadIdx.x) + it * kBlk, NCH - 1);
            const int pix = idx / (CIN / 8), c8 = idx - pix * (CIN / 8);
            const int gy = y0 + pix / PW - 1, gx = x0 + pix % PW - 1;
            const bool ok = gy >= 0 && gy < H && gx >= 0 && gx < W;
            if constexpr (XIN) {
                const int64_t e = ok ? ((int64_t(n) * (H / 2) + (gy >> 1)) * (W / 2) + (gx >> 1)) * CIN + 8 * c8 : 0;
                v[it] = *reinterpret_cast<const uint4 *>(in + e);
                vm[it] = *reinterpret_cast<const uint2 *>(xmask + e);
            } else {
                const uint4 t = *reinterpret_cast<const uint4 *>(
                    in + (ok ? ((int64_t(n) * H + gy) * W + gx) * CIN + 8 * c8 : int64_t(0)));
                v[it] = ok ? t : make_uint4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int it = 0; it < NR; ++it) {
            const int idx = int(threadIdx.x) + it * kBlk;
            if (idx < NCH) {
                const int pix = idx / (CIN / 8), c8 = idx - pix * (CIN / 8);
                uint4 t = v[it];
                if constexpr (XIN) {
                    const int gy = y0 + pix / PW - 1, gx = x0 + pix % PW - 1;
                    const bool ok = gy >= 0 && gy < H && gx >= 0 && gx < W;
                    t = ok ? expand8(t, vm[it], ((gy & 1) << 1) | (gx & 1)) : make_uint4(0, 0, 0, 0);
                }
                *reinterpret_cast<uint4 *>(patch + (pix / PW) * RS + (pix % PW) * PS + 8 * c8) = t;
            }
        }
    }
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    // wavefront's first channel, and first quad row (pairs of pixel rows) of the tile
    const int cw = blockIdx.y * BN + (wv / PG) * (BN / CG);
    const int qr0 = (wv % PG) * (8 * MT / TW);
    const int r16 = lane & 15, kq = lane >> 4;
    // patch pixel (before the tap shift) of this lane's row in each M tile:
    // row 16 r + r16 is quad 4 r + r16 / 4, position r16 mod 4
    int abase[MT];
#pragma unroll
    for (int r = 0; r < MT; ++r) {
        const int ql = 4 * r + (r16 >> 2), sub = r16 & 3;
        const int y = 2 * (qr0 + ql / QW) + (sub >> 1), x = 2 * (ql % QW) + (sub & 1);
        abase[r] = (y + 1) * RS + (x + 1) * PS + 8 * kq;
    }
    const u16 *wrow[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) wrow[c] = wt + int64_t(cw + 16 * c + r16) * (9 * CIN) + 8 * kq;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int r = 0; r < MT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    Frag bcur[NT], bnext[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) bcur[c].u = *reinterpret_cast<const uint4 *>(wrow[c]);
    __syncthreads();
#pragma unroll 1
    for (int kk = 0; kk < NK; ++kk) {
        if (kk + 1 < NK) {
#pragma unroll
            for (int c = 0; c < NT; ++c) bnext[c].u = *reinterpret_cast<const uint4 *>(wrow[c] + (kk + 1) * 32);
        }
        const int tap = kk / KPT, ci0 = (kk - tap * KPT) * 32;
        const int shift = (tap / 3 - 1) * RS + (tap % 3 - 1) * PS + ci0;
        Frag a[MT];
#pragma unroll
        for (int r = 0; r < MT; ++r) a[r].u = *reinterpret_cast<const uint4 *>(patch + abase[r] + shift);
#pragma unroll
        for (int r = 0; r < MT; ++r)
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                // the expanding epilogue takes the transposed product: four
                // consecutive channels of one pixel per lane
                if constexpr (EPI == kEpiExpand)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bcur[c].v, a[r].v, acc[r][c], 0, 0, 0);
                else
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r].v, bcur[c].v, acc[r][c], 0, 0, 0);
            }
#pragma unroll
        for (int c = 0; c < NT; ++c) bcur[c] = bnext[c];
    }
    if constexpr (EPI == kEpiExpand) {
        // input gradient of a pooled layer: this layer's output grid is the
        // pooled grid of the one below; each value, times a quarter, goes to
        // the 2 x 2 pixels whose ReLU was active (mask_out holds the masks of
        // the layer below, read here).  This lane holds channels
        // cw + 16 c + 4 kq .. + 3 of pixel row 16 r + r16 of the tile (quad
        // 4 r + r16 / 4, position r16 mod 4): one 4-byte mask load and four
        // 8-byte stores per tile.
#pragma unroll
        for (int r = 0; r < MT; ++r) {
            const int ql = 4 * r + (r16 >> 2), pos = r16 & 3;
            const int qy = y0 / 2 + qr0 + ql / QW, qx = x0 / 2 + ql % QW;
            const int y = 2 * qy + (pos >> 1), x = 2 * qx + (pos & 1);
            const int64_t pp = (int64_t(n) * H + y) * W + x;
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const int co0 = cw + 16 * c + 4 * kq;
                const uint32_t m4 = *reinterpret_cast<const uint32_t *>(mask_out + pp * Cout + co0);
                u16 h[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) h[i] = f2bf(0.25f * bf2f(f2bf(acc[r][c][i])));
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    u16 v[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = (m4 >> (8 * i + d)) & 1u ? h[i] : u16(0);
                    const int64_t o = ((int64_t(n) * 2 * H + 2 * y + (d >> 1)) * (2 * W) + 2 * x + (d & 1)) * Cout + co0;
                    *reinterpret_cast<uint2 *>(out + o) = make_uint2(uint32_t(v[0]) | (uint32_t(v[1]) << 16),
                                                                     uint32_t(v[2]) | (uint32_t(v[3]) << 16));
                }
            }
        }
        return;
    }
    // epilogue: this lane holds quad 4 r + kq of M tile r, channel column
    // r16 of N tile c
#pragma unroll
    for (int r = 0; r < MT; ++r) {
        const int ql = 4 * r + kq;
        const int qy = y0 / 2 + qr0 + ql / QW, qx = x0 / 2 + ql % QW;  // pooled coordinates
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int co = cw + 16 * c + r16;
            // raw input gradients carry no bias
            const float bv = EPI == kEpiRaw ? 0.0f : bias[co];
            if constexpr (EPI == kEpiPool) {
                const int64_t q = (int64_t(n) * (H / 2) + qy) * (W / 2) + qx;
                float s4 = 0.0f;
                unsigned m = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float a = bf2f(f2bf(fmaxf(acc[r][c][i] + bv, 0.0f)));
                    s4 += a;
                    m |= (a > 0.0f ? 1u : 0u) << i;
                }
                out[q * Cout + co] = f2bf(0.25f * s4);
                mask_out[q * Cout + co] = uint8_t(m);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int y = 2 * qy + (i >> 1), x = 2 * qx + (i & 1);
                    const float v = acc[r][c][i] + bv;
                    out[((int64_t(n) * H + y) * W + x) * Cout + co] = f2bf(EPI == kEpiRaw ? v : fmaxf(v, 0.0f));
                }
            }
        }
    }
}

// Register target of four waves per SIMD (three for 8 x 32 tiles, whose
// 49 KB patch leaves room for three workgroups per CU); with 128 input
// channels the patch is 49 KB too, and that variant keeps its registers
// (measured faster than squeezed).
template <int CIN, int TW, int BN, int EPI, int MT = 4, bool XIN = false>
__global__ __launch_bounds__(kBlk) __attribute__((amdgpu_waves_per_eu(TW == 32 ? 3 : 4))) void k_conv_lds(
    const u16 *in, const u16 *wt, const float *bias, u16 *out, uint8_t *mask_out, int B, int H, int W, int Cout,
    const uint8_t *xmask = nullptr) {
    conv_lds_body<CIN, TW, BN, EPI, MT, XIN>(in, wt, bias, out, mask_out, B, H, W, Cout, xmask);
}

template <int TW, int BN, int EPI, int MT = 4>
__global__ __launch_bounds__(kBlk) void k_conv_lds128(const u16 *in, const u16 *wt, const float *bias, u16 *out,
                                                     uint8_t *mask_out, int B, int H, int W, int Cout) {
    conv_lds_body<128, TW, BN, EPI, MT>(in, wt, bias, out, mask_out, B, H, W, Cout);
}

// 256 input channels (the input gradient of the last layer): a 53 KB patch
template <int TW, int BN, int EPI>
__global__ __launch_bounds__(kBlk) void k_conv_lds256(const u16 *in, const u16 *wt, const float *bias, u16 *out,
                                                     uint8_t *mask_out, int B, int H, int W, int Cout) {
    conv_lds_body<256, TW, BN, EPI, 4>(in, wt, bias, out, mask_out, B, H, W, Cout);
}

// The staged-patch kernel takes layers with 32, 64 or 128 input channels
// whose 8 x TW tiles and 64-channel blocks divide the layer exactly; layers
// with a multiple of 128 output channels take 128-channel blocks (one
// staged patch feeds twice the MFMA work).
inline int conv_lds_tw(int H, int W, int Cin, int Cout) {
    if (!(Cin == 32 || Cin == 64 || Cin == 128) || H % 8 != 0 || Cout % 64 != 0) return 0;
    return W % 16 == 0 ? 16 : (W % 8 == 0 ? 8 : 0);
}

template <int EPI, int TW, int BN>
void launch_conv_lds_bn(hipStream_t st, const u16 *in, const u16 *wt, const float *bias, u16 *out, uint8_t *mask,
                        int B, int H, int Cin, int Cout) {
    // 8 x 16 tiles: each wavefront takes all 128 pixels and BN / 4 channels
    // (half the weight loads per MFMA of 64-pixel wavefronts over BN / 2)
    constexpr int MT = TW >= 16 ? 8 : 4;
    const dim3 g(unsigned(B * (H / 8) * (H / TW)), unsigned(Cout / BN));
    if (Cin == 32)
        hipLaunchKernelGGL((k_conv_lds<32, TW, BN, EPI, MT>), g, dim3(kBlk), 0, st, in, wt, bias, out, mask, B, H, H, Cout);
    else if (Cin == 64)
        hipLaunchKernelGGL((k_conv_lds<64, TW, BN, EPI, MT>), g, dim3(kBlk), 0, st, in, wt, bias, out, mask, B, H, H, Cout);
    else
        hipLaunchKernelGGL((k_conv_lds128<TW, BN, EPI, MT>), g, dim3(kBlk), 0, st, in, wt, bias, out, mask, B, H, H, Cout);
}

template <int EPI>
void launch_conv_lds(hipStream_t st, int tw, const u16 *in, const u16 *wt, const float *bias, u16 *out,
                     uint8_t *mask, int B, int H, int Cin, int Cout) {
    const bool wide = Cout % 128 == 0;
    // (8 x 32 tiles for the 32-channel layer: 119 against 108 us)
    if (tw == 16 && wide) launch_conv_lds_bn<EPI, 16, 128>(st, in, wt, bias, out, mask, B, H, Cin, Cout);
    else if (tw == 16) launch_conv_lds_bn<EPI, 16, 64>(st, in, wt, bias, out, mask, B, H, Cin, Cout);
    else if (wide) launch_conv_lds_bn<EPI, 8, 128>(st, in, wt, bias, out, mask, B, H, Cin, Cout);
    else launch_conv_lds_bn<EPI, 8, 64>(st, in, wt, bias, out, mask, B, H, Cin, Cout);
}

constexpr int kConvWM = 4, kConvWN = 4;  // 64 pixels x 64 channels per wavefront

// four wavefronts of WM * 16 pixels per workgroup along x, WN * 16 channels along y
inline dim3 conv_grid(int64_t npix, int cout) {
    return dim3(unsigned((npix + 64 * kConvWM - 1) / (64 * kConvWM)), unsigned((cout + 16 * kConvWN - 1) / (16 * kConvWN)));
}

// ------------------------------------------------------- weight gradient
// dw[co, n] = sum_p dout[p, co] * in[shift(p, tap(n)), ci(n)], n = tap * Cin
// + ci (the [Cout][9][Cin] weight layout flattened), split over pixel
// ranges: partial[split][co][n] (FP32), summed later in a fixed order.
// Workgroup tile: 64 output channels x 288 columns (a multiple of 288 =
// 9 x 32 for every Cin), so dout is read once per 288 columns and the input
// patches once per 64 output channels; 64 pixels of reduction per LDS
// stage.  Per stage lane l of every wavefront stages pixel l: dout channels
// 16 w .. 16 w + 15 and input chunks 9 w .. 9 w + 8 (eight columns each; Cin
// is a power of two >= 32, so a chunk never straddles a tap), with one
// division of the pixel index per stage.  Both tiles are stored in their
// natural [pixel][channel] order with 16-byte stores and read back as MFMA
// operands with the transposing LDS read (ds_read_b64_tr_b16): within a
// group of 16 lanes, lane L addressing T[k0 + L / 4][m0 + 4 (L mod 4)] makes
// lane i receive T[k0 + k][m0 + i], k = 0..3 -- four consecutive reduction
// elements of row m0 + i, half of an MFMA fragment.  Wavefront w computes
// 32 channels x 144 columns (2 x 9 tiles of 16 x 16).  The workgroups of
// the first column tile also sum dout over their pixels: the bias gradient.
// (64 x 64 tiles, which re-read dout for every 64 columns, took 276 us per
// layer on average against 147.)
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4s lds_v4s;

constexpr int kWwN = 288;          // columns per workgroup
constexpr int kWwXS = kWwN + 8;    // u16 per staged input pixel row: 592 B, 16-byte aligned
constexpr int kWwDS = 64 + 8;      // u16 per staged dout pixel row

template <int S>
__device__ inline bf16x8 tr_frag_s(const u16 *tile, int k0, int m0, int lane16) {
    const u16 *p0 = tile + (k0 + (lane16 >> 2)) * S + m0 + 4 * (lane16 & 3);
    union {
        v4s h[2];
        bf16x8 v;
    } u;
    u.h[0] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)(p0));
    u.h[1] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)(p0 + 4 * S));
    return u.v;
}

__global__ __launch_bounds__(kBlk) void k_conv_wgrad_wide(const u16 *in, const u16 *dout, float *partial,
                                                         float *bias_partial, int B, int H, int W, int Cin,
                                                         int Cout, int pix_per_split) {
    __shared__ __align__(16) u16 sd[64 * kWwDS];  // [pixel][co]
    __shared__ __align__(16) u16 sx[64 * kWwXS];  // [pixel][n]
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int N = 9 * Cin;
    const int co_t = blockIdx.x * 64, n_t = blockIdx.y * kWwN;
    const int split = blockIdx.z;
    const int npix = B * H * W;
    const int pbeg = split * pix_per_split;
    const int pend = min(pbeg + pix_per_split, npix);
    const int r16 = lane & 15, kq = lane >> 4;
    const int wco = (wv >> 1) * 32, wn = (wv & 1) * 144;
    const bool do_bias = blockIdx.y == 0;
    const int cshift = __builtin_ctz(unsigned(Cin));
    f32x4 acc[2][9];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) bsum[e] = 0.0f;
    uint4 rd[2], rx[9];
    auto gload = [&](int q0) {
        const int p = q0 + lane;
        const bool pin = p < pend;
        const int pp = pin ? p : 0;
        const int x = pp % W, t = pp / W, y = t % H, n = t / H;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int co = co_t + 16 * wv + 8 * h;
            const bool dok = pin && co < Cout;
            // unconditional loads from valid addresses, masked afterwards
            const uint4 v = *reinterpret_cast<const uint4 *>(dout + (dok ? int64_t(pp) * Cout + co : 0));
            rd[h] = dok ? v : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int nn = n_t + 8 * (9 * wv + j);
            const int tap = nn >> cshift, ci = nn & (Cin - 1);
            const int sy = y + tap / 3 - 1, sx2 = x + tap % 3 - 1;
            const bool xok = pin && sy >= 0 && sy < H && sx2 >= 0 && sx2 < W;
            const uint4 v =
                *reinterpret_cast<const uint4 *>(in + (xok ? (int64_t((n * H + sy) * W + sx2) << cshift) + ci : 0));
            rx[j] = xok ? v : make_uint4(0, 0, 0, 0);
        }
    };
    if (pbeg < pend) gload(pbeg);
    for (int q0 = pbeg; q0 < pend; q0 += 64) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            *reinterpret_cast<uint4 *>(sd + lane * kWwDS + 16 * wv + 8 * h) = rd[h];
            if (do_bias) {
                const u16 *e8 = reinterpret_cast<const u16 *>(&rd[h]);
#pragma unroll
                for (int e = 0; e < 8; ++e) bsum[8 * h + e] += bf2f(e8[e]);
            }
        }
#pragma unroll
        for (int j = 0; j < 9; ++j) *reinterpret_cast<uint4 *>(sx + lane * kWwXS + 8 * (9 * wv + j)) = rx[j];
        __syncthreads();
        if (q0 + 64 < pend) gload(q0 + 64);  // next stage in flight during the MFMAs
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 a[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) a[r] = tr_frag_s<kWwDS>(sd, ks * 32 + 8 * kq, wco + r * 16, r16);
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const bf16x8 bb = tr_frag_s<kWwXS>(sx, ks * 32 + 8 * kq, wn + c * 16, r16);
#pragma unroll
                for (int r = 0; r < 2; ++r)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], bb, acc[r][c], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D: rows = co (4 kq + i), column = n (r16)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const int n = n_t + wn + c * 16 + r16;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = co_t + wco + r * 16 + 4 * kq + i;
                if (co < Cout && n < N) partial[(int64_t(split) * Cout + co) * N + n] = acc[r][c][i];
            }
        }
    if (do_bias) {  // uniform per workgroup
        // lane l summed pixel l of every stage: butterfly over the 64 lanes
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            float v = bsum[e];
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
            bsum[e] = v;
        }
        if (lane == 0) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int co = co_t + 16 * wv + e;
                if (co < Cout) bias_partial[int64_t(split) * Cout + co] = bsum[e];
            }
        }
    }
}

// Weight gradient over 8 x 8 pixel tiles (layers whose sides are multiples
// of 8): per tile the 64 pixels' dout rows and the input of the tile with
// its one-pixel halo (10 x 10 pixels, 32 input channels) are staged once;
// the operand of tap (ty, tx) for the tile's pixel row y is then the staged
// halo row y + ty from column tx on -- eight consecutive staged pixels, so
// the transposing LDS read takes it as it takes a dout row.  Each input
// value is loaded once per tile instead of once per tap.  Workgroup tile:
// 64 output channels x (9 taps x 32 input channels); wavefront w computes
// 32 channels x nine of the eighteen 16-column tiles (tile ct: tap ct / 2,
// channels 16 (ct mod 2) ..).  Splits are runs of tiles; partial[split][co]
// [n] as for the wide kernel, bias partials from the workgroups of the
// first channel block (fixed-order reductions).
constexpr int kWhS = 48;     // u16 per staged halo pixel: 32 channels + pad (conflict-free transposed reads)
constexpr int kWhPix = 100;  // 10 x 10 staged pixels

// XD: dout is the pooled gradient [B][H/2][W/2][Cout] with the ReLU masks
// dmask of the layer (expanded while staging) instead of the full-resolution one.
template <bool XD>
__global__ __launch_bounds__(kBlk) __attribute__((amdgpu_waves_per_eu(XD ? 2 : 3))) void k_conv_wgrad_halo(
    const u16 *in, const u16 *dout, const uint8_t *dmask, float *partial, float *bias_partial, int B, int H, int W,
    int Cin, int Cout, int tiles_per_split) {
    __shared__ __align__(16) u16 sd[64 * kWwDS];     // [tile pixel][co]
    __shared__ __align__(16) u16 sx[kWhPix * kWhS];  // [halo pixel][ci]
    __shared__ float bred[kBlk / 64][64];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int N = 9 * Cin;
    const int co_t = blockIdx.x * 64, ci_t = blockIdx.y * 32;
    const int split = blockIdx.z;
    const int tx_n = W >> 3, ty_n = H >> 3;
    const int ntiles = B * ty_n * tx_n;
    const int tbeg = split * tiles_per_split;
    const int tend = min(tbeg + tiles_per_split, ntiles);
    const int r16 = lane & 15, kq = lane >> 4;
    const int wco = (wv >> 1) * 32, wct = (wv & 1) * 9;
    const bool do_bias = blockIdx.y == 0;
    f32x4 acc[2][9];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) bsum[e] = 0.0f;
    // staging: dout chunk q = tid + 256 i is tile pixel q / 8, channels
    // co_t + 8 (q mod 8); halo chunk h = tid + 256 i (h < 400) is halo pixel
    // h / 4, channels ci_t + 8 (h mod 4)
    uint4 rd[2], rx[2];
    uint2 rm[2];  // XD: the mask bytes of rd's channels
    auto gload = [&](int t) {
        const int txi = t % tx_n, rr = t / tx_n, tyi = rr % ty_n, n = rr / ty_n;
        const int y0 = 8 * tyi, x0 = 8 * txi;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int q = tid + kBlk * i, pix = q >> 3;
            if constexpr (XD) {
                const int64_t pp = (int64_t(n) * (H / 2) + ((y0 + (pix >> 3)) >> 1)) * (W / 2) + ((x0 + (pix & 7)) >> 1);
                rd[i] = *reinterpret_cast<const uint4 *>(dout + pp * Cout + co_t + 8 * (q & 7));
                rm[i] = *reinterpret_cast<const uint2 *>(dmask + pp * Cout + co_t + 8 * (q & 7));
            } else {
                const int64_t p = (int64_t(n) * H + y0 + (pix >> 3)) * W + x0 + (pix & 7);
                rd[i] = *reinterpret_cast<const uint4 *>(dout + p * Cout + co_t + 8 * (q & 7));
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            // unconditional loads from valid addresses, zeroed off the image
            const int h = tid + kBlk * i, hp = min(h >> 2, kWhPix - 1);
            const int y = y0 + hp / 10 - 1, x = x0 + hp % 10 - 1;
            const bool ok = h < 4 * kWhPix && y >= 0 && y < H && x >= 0 && x < W;
            const int64_t pi = ok ? (int64_t(n) * H + y) * W + x : 0;
            const uint4 v = *reinterpret_cast<const uint4 *>(in + pi * Cin + ci_t + 8 * (h & 3));
            rx[i] = ok ? v : make_uint4(0, 0, 0, 0);
        }
    };
    if (tbeg < tend) gload(tbeg);
    for (int t = tbeg; t < tend; ++t) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int q = tid + kBlk * i;
            // (tile origins are even: the sub-pixel is the tile pixel's parity)
            if constexpr (XD) rd[i] = expand8(rd[i], rm[i], (((q >> 6) & 1) << 1) | ((q >> 3) & 1));
            *reinterpret_cast<uint4 *>(sd + (q >> 3) * kWwDS + 8 * (q & 7)) = rd[i];
            if (do_bias) {
                const u16 *e8 = reinterpret_cast<const u16 *>(&rd[i]);
#pragma unroll
                for (int e = 0; e < 8; ++e) bsum[e] += bf2f(e8[e]);
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int h = tid + kBlk * i;
            if (h < 4 * kWhPix) *reinterpret_cast<uint4 *>(sx + (h >> 2) * kWhS + 8 * (h & 3)) = rx[i];
        }
        __syncthreads();
        if (t + 1 < tend) gload(t + 1);  // next tile in flight during the MFMAs
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int k0 = ks * 32 + 8 * kq;  // tile pixels k0 .. k0 + 7: row k0 / 8
            bf16x8 a[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) a[r] = tr_frag_s<kWwDS>(sd, k0, wco + r * 16, r16);
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const int ct = wct + c, tap = ct >> 1;
                const int hrow = ((k0 >> 3) + tap / 3) * 10 + tap % 3;
                const bf16x8 bb = tr_frag_s<kWhS>(sx, hrow, 16 * (ct & 1), r16);
#pragma unroll
                for (int r = 0; r < 2; ++r)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], bb, acc[r][c], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D: rows = co (4 kq + i), column = r16 of tile ct
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const int ct = wct + c;
            const int n = (ct >> 1) * Cin + ci_t + 16 * (ct & 1) + r16;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = co_t + wco + r * 16 + 4 * kq + i;
                partial[(int64_t(split) * Cout + co) * N + n] = acc[r][c][i];
            }
        }
    if (do_bias) {  // uniform per workgroup
        // thread tid summed channels co_t + 8 (tid mod 8) ..: lanes of equal
        // tid mod 8 within the wavefront, then the four wavefronts in order
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float v = bsum[e];
#pragma unroll
            for (int o = 8; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
            bsum[e] = v;
        }
        if (lane < 8) {
#pragma unroll
            for (int e = 0; e < 8; ++e) bred[wv][8 * lane + e] = bsum[e];
        }
        __syncthreads();
        if (tid < 64) {
            float v = 0.0f;
#pragma unroll
            for (int w = 0; w < kBlk / 64; ++w) v += bred[w][tid];
            bias_partial[int64_t(split) * Cout + co_t + tid] = v;
        }
    }
}

// Fixed-order sum of split partials: wavefront w of a workgroup sums the
// splits k = w (mod 4) of 64 consecutive outputs in split order, and the
// four are combined as (s0 + s1) + (s2 + s3) -- a quarter of the dependent
// loads per lane of one running sum per output.
__global__ __launch_bounds__(kBlk) void k_sum_splits(const float *partial, float *out, int64_t n, int splits) {
    __shared__ float red[kBlk / 64][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = int64_t(blockIdx.x) * 64 + lane;
    const bool ok = i < n;
    const int64_t ii = ok ? i : 0;
    float s = 0.0f;
#pragma unroll 8
    for (int k = w; k < splits; k += 4) s += partial[int64_t(k) * n + ii];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && ok) out[i] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Weight gradient of the one-channel first layer: partials [split][co][10]
// (9 taps, then the bias).  Wavefront w of a workgroup handles channels
// 8 w .. 8 w + 7 (workgroups along y cover further groups).
__device__ inline float wave_sum_f(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Backward of the fused first layer: from the pooled gradient dpool, the
// conv-output gradient of sub-pixel d is bf16(dpool / 4) where the forward
// pass's BF16 ReLU output was positive (its mask bits), else 0; it is
// multiplied into the 9 image taps and the bias.  Each wavefront takes
// kC1Cpw channels (40 accumulators per lane, 90 registers: five wavefronts per SIMD, where
// eight channels needed 130 registers and got three); pooled pixels of a
// split are strided over the lanes; a fixed wavefront reduction combines
// the lanes.
constexpr int kC1Cpw = 4;

__global__ __launch_bounds__(kBlk) void k_conv1_bwd(const uint8_t *x, const uint32_t *mask, const u16 *dpool,
                                                   float *partial, int B, int H, int W, int C,
                                                   int64_t q_per_split) {
    const int lane = threadIdx.x & 63;
    const int grp = (blockIdx.y * (kBlk / 64)) + (threadIdx.x >> 6);
    if (grp * kC1Cpw >= C) return;  // whole wavefronts leave together
    const int Ho = H / 2, Wo = W / 2;
    const int64_t nq = int64_t(B) * Ho * Wo;
    const int64_t b0 = int64_t(blockIdx.x) * q_per_split;
    const int64_t b1 = b0 + q_per_split < nq ? b0 + q_per_split : nq;
    // the mask word of eight channels holds this group's 16 bits at msh
    const int mw = grp * kC1Cpw / 8, msh = (grp * kC1Cpw) % 8 * 4;
    float acc[kC1Cpw][10];
#pragma unroll
    for (int e = 0; e < kC1Cpw; ++e)
#pragma unroll
        for (int k = 0; k < 10; ++k) acc[e][k] = 0.0f;
    for (int64_t q = b0 + lane; q < b1; q += 64) {
        const uint2 gv = *reinterpret_cast<const uint2 *>(dpool + q * C + grp * kC1Cpw);
        const u16 *gh = reinterpret_cast<const u16 *>(&gv);
        const uint32_t mb = mask[q * (C / 8) + mw] >> msh;
        int xo, yo;
        int64_t n;
        split_pooled(q, Wo, Ho, xo, yo, n);
        float v[4][4];
        conv1_patch(x, H, W, n, yo, xo, v);
#pragma unroll
        for (int e = 0; e < kC1Cpw; ++e) {
            const float g = bf2f(f2bf(0.25f * bf2f(gh[e])));
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int dy = d >> 1, dx = d & 1;
                const float da = (mb >> (4 * e + d)) & 1u ? g : 0.0f;
#pragma unroll
                for (int t = 0; t < 9; ++t) acc[e][t] = fmaf(da, v[dy + t / 3][dx + t % 3], acc[e][t]);
                acc[e][9] += da;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < kC1Cpw; ++e)
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const float t = wave_sum_f(acc[e][k]);
            if (lane == 0) partial[(int64_t(blockIdx.x) * C + grp * kC1Cpw + e) * 10 + k] = t;
        }
}

// The same backward walking down pooled rows (images whose pooled width is
// a multiple of 64 and pooled height a multiple of kC1Rows): lane l of a
// split owns pooled column 64 chunk + l of kC1Rows consecutive pooled rows
// of one image; the 4 x 4 image patch of the next row shares two rows with
// the current one, so each step loads two new patch rows (eight bytes) and
// no pixel index is divided.  Same arithmetic per pooled pixel; splits are
// (row block, column chunk), kSplitPix / 4 pooled pixels each.
constexpr int kC1Rows = 32;

__global__ __launch_bounds__(kBlk) void k_conv1_bwd_rows(const uint8_t *x, const uint32_t *mask, const u16 *dpool,
                                                        float *partial, int B, int H, int W, int C) {
    const int lane = threadIdx.x & 63;
    const int grp = (blockIdx.y * (kBlk / 64)) + (threadIdx.x >> 6);
    if (grp * kC1Cpw >= C) return;  // whole wavefronts leave together
    const int Ho = H / 2, Wo = W / 2, nch = Wo / 64;
    const int chunk = int(blockIdx.x) % nch, rb = int(blockIdx.x) / nch;
    const int n = rb * kC1Rows / Ho, yo0 = rb * kC1Rows % Ho;
    const int xo = 64 * chunk + lane;
    const int mw = grp * kC1Cpw / 8, msh = (grp * kC1Cpw) % 8 * 4;
    const uint8_t *img = x + int64_t(n) * H * W;
    // patch column c: image column 2 xo - 1 + c (clamped; off the image its values are zeroed)
    int cx[4];
    float con[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int sx = 2 * xo - 1 + c;
        cx[c] = min(max(sx, 0), W - 1);
        con[c] = sx >= 0 && sx < W ? 1.0f : 0.0f;
    }
    auto load_row = [&](int sy, float *row) {
        const int cy = min(max(sy, 0), H - 1);
        const float on = sy >= 0 && sy < H ? 1.0f : 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c) row[c] = float(img[int64_t(cy) * W + cx[c]]) * (on * con[c]);
    };
    float acc[kC1Cpw][10];
#pragma unroll
    for (int e = 0; e < kC1Cpw; ++e)
#pragma unroll
        for (int k = 0; k < 10; ++k) acc[e][k] = 0.0f;
    float v[4][4];
#pragma unroll
    for (int r = 0; r < 2; ++r) load_row(2 * yo0 - 1 + r, v[r]);
    for (int yo = yo0; yo < yo0 + kC1Rows; ++yo) {
        load_row(2 * yo + 1, v[2]);
        load_row(2 * yo + 2, v[3]);
        const int64_t q = (int64_t(n) * Ho + yo) * Wo + xo;
        const uint2 gv = *reinterpret_cast<const uint2 *>(dpool + q * C + grp * kC1Cpw);
        const u16 *gh = reinterpret_cast<const u16 *>(&gv);
        const uint32_t mb = mask[q * (C / 8) + mw] >> msh;
#pragma unroll
        for (int e = 0; e < kC1Cpw; ++e) {
            const float g = bf2f(f2bf(0.25f * bf2f(gh[e])));
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int dy = d >> 1, dx = d & 1;
                const float da = (mb >> (4 * e + d)) & 1u ? g : 0.0f;
#pragma unroll
                for (int t = 0; t < 9; ++t) acc[e][t] = fmaf(da, v[dy + t / 3][dx + t % 3], acc[e][t]);
                acc[e][9] += da;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            v[0][c] = v[2][c];
            v[1][c] = v[3][c];
        }
    }
#pragma unroll
    for (int e = 0; e < kC1Cpw; ++e)
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const float t = wave_sum_f(acc[e][k]);
            if (lane == 0) partial[(int64_t(blockIdx.x) * C + grp * kC1Cpw + e) * 10 + k] = t;
        }
}

// ------------------------------------------------------ pooling and GAP
__global__ __launch_bounds__(kBlk) void k_gap_fwd(const u16 *in, float *out, int B, int HW, int C) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (i >= int64_t(B) * C) return;
    const int c = int(i % C);
    const int64_t n = i / C;
    float s = 0.0f;
    // unrolled so the loads of eight pixels are in flight together (the sum
    // keeps its order)
#pragma unroll 8
    for (int p = 0; p < HW; ++p) s += bf2f(in[(n * HW + p) * C + c]);
    out[i] = s / float(HW);
}

// Gradient of the last conv output: dg / HW where its ReLU output is
// positive.  One thread per pixel and eight channels (C is a multiple of
// 8): 16-byte loads and stores, one index division per eight values.
__global__ __launch_bounds__(kBlk) void k_gap_bwd_relu(const float *dg, const u16 *act, u16 *dact, int B, int HW,
                                                      int C) {
    const int64_t t = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    const int64_t total8 = int64_t(B) * HW * (C / 8);
    if (t >= total8) return;
    const int64_t i = 8 * t;  // first of the eight elements
    int c0;
    int64_t n;
    if (i <= 0x7FFFFFFF) {  // 32-bit division where the index fits
        const uint32_t u = uint32_t(i);
        c0 = int(u % uint32_t(C));
        n = int64_t(u / uint32_t(HW * C));
    } else {
        c0 = int(i % C);
        n = i / (int64_t(HW) * C);
    }
    const uint4 a = *reinterpret_cast<const uint4 *>(act + i);
    const u16 *ah = reinterpret_cast<const u16 *>(&a);
    u16 o[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float g = dg[n * C + c0 + e] / float(HW);
        o[e] = f2bf(bf2f(ah[e]) > 0.0f ? g : 0.0f);
    }
    *reinterpret_cast<uint4 *>(dact + i) = *reinterpret_cast<const uint4 *>(o);
}

// ---------------------------------------------------------- dense layers
// y[n, o] = act(b[o] + sum_i w[o, i] x[n, i]), summed in the order i = 0,
// 1, ...  A workgroup computes 8 samples x 64 outputs (two outputs per
// thread), staging 128-wide slices of x and w in LDS with coalesced row
// loads (rows padded by one float against bank conflicts); the small tile
// gives a few hundred workgroups for a batch of 512, and the wide slices
// few staging round trips (two for 256 inputs).
constexpr int kFcN = 8, kFcO = 64, kFcI = 128;

__global__ __launch_bounds__(kBlk) void k_fc_fwd(const float *x, const float *w, const float *b, float *y, int B,
                                                int In, int Out, int relu) {
    __shared__ float xs[kFcN][kFcI + 1];
    __shared__ float ws[kFcO][kFcI + 1];
    const int n0 = blockIdx.y * kFcN, o0 = blockIdx.x * kFcO;
    const int nl = threadIdx.x >> 5, og = threadIdx.x & 31;  // sample, outputs og and og + 32
    float s[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int o = o0 + og + 32 * j;
        s[j] = o < Out ? b[o] : 0.0f;
    }
    for (int i0 = 0; i0 < In; i0 += kFcI) {
        // fixed trip counts, unrolled; a slice inside the matrices (uniform
        // over the workgroup) loads without guards, so every staging load is
        // in flight before the first LDS store waits
        static_assert((kFcN * kFcI) % kBlk == 0 && (kFcO * kFcI) % kBlk == 0, "whole staging rounds");
        const bool inside = n0 + kFcN <= B && o0 + kFcO <= Out && i0 + kFcI <= In;
        if (inside) {
            float xv[kFcN * kFcI / kBlk], wv[kFcO * kFcI / kBlk];
#pragma unroll
            for (int t = 0; t < kFcN * kFcI / kBlk; ++t) {
                const int e = int(threadIdx.x) + t * kBlk;
                xv[t] = x[int64_t(n0 + e / kFcI) * In + i0 + e % kFcI];
            }
#pragma unroll
            for (int t = 0; t < kFcO * kFcI / kBlk; ++t) {
                const int e = int(threadIdx.x) + t * kBlk;
                wv[t] = w[int64_t(o0 + e / kFcI) * In + i0 + e % kFcI];
            }
#pragma unroll
            for (int t = 0; t < kFcN * kFcI / kBlk; ++t) {
                const int e = int(threadIdx.x) + t * kBlk;
                xs[e / kFcI][e % kFcI] = xv[t];
            }
#pragma unroll
            for (int t = 0; t < kFcO * kFcI / kBlk; ++t) {
                const int e = int(threadIdx.x) + t * kBlk;
                ws[e / kFcI][e % kFcI] = wv[t];
            }
        } else {
            for (int e = threadIdx.x; e < kFcN * kFcI; e += kBlk) {
                const int r = e / kFcI, c = e % kFcI;
                const int n = n0 + r, i = i0 + c;
                xs[r][c] = (n < B && i < In) ? x[int64_t(n) * In + i] : 0.0f;
            }
            for (int e = threadIdx.x; e < kFcO * kFcI; e += kBlk) {
                const int r = e / kFcI, c = e % kFcI;
                const int o = o0 + r, i = i0 + c;
                ws[r][c] = (o < Out && i < In) ? w[int64_t(o) * In + i] : 0.0f;
            }
        }
        __syncthreads();
        const int ni = min(kFcI, In - i0);
        if (ni == kFcI) {
            // full slice: unrolled, so the LDS reads are issued ahead of the
            // dependent multiply-add chains
#pragma unroll 16
            for (int c = 0; c < kFcI; ++c) {
                const float xv = xs[nl][c];
#pragma unroll
                for (int j = 0; j < 2; ++j) s[j] = fmaf(ws[og + 32 * j][c], xv, s[j]);
            }
        } else {
            for (int c = 0; c < ni; ++c) {
                const float xv = xs[nl][c];
#pragma unroll
                for (int j = 0; j < 2; ++j) s[j] = fmaf(ws[og + 32 * j][c], xv, s[j]);
            }
        }
        __syncthreads();
    }
    const int n = n0 + nl;
    if (n >= B) return;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int o = o0 + og + 32 * j;
        if (o < Out) y[int64_t(n) * Out + o] = relu ? fmaxf(s[j], 0.0f) : s[j];
    }
}

inline dim3 fc_grid(int B, int Out) { return dim3(unsigned((Out + kFcO - 1) / kFcO), unsigned((B + kFcN - 1) / kFcN)); }

// dx[n, i] = sum_o w[o, i] dy[n, o], times the ReLU mask of x when given
__global__ __launch_bounds__(kBlk) void k_fc_bwd_data(const float *dy, const float *w, const float *xact,
                                                     float *dx, int B, int In, int Out) {
    const int64_t t = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (t >= int64_t(B) * In) return;
    const int i = int(t % In);
    const int64_t n = t / In;
    float s = 0.0f;
#pragma unroll 8
    for (int o = 0; o < Out; ++o) s = fmaf(w[int64_t(o) * In + i], dy[n * Out + o], s);
    if (xact && !(xact[t] > 0.0f)) s = 0.0f;
    dx[t] = s;
}

// dw[o, i] = sum_n dy[n, o] x[n, i]; db[o] = sum_n dy[n, o] (column In).
// Wavefront w of a workgroup sums the samples n = w (mod 4) of 64
// consecutive outputs in sample order (the bias column multiplies by one);
// the four are combined as (s0 + s1) + (s2 + s3).
__global__ __launch_bounds__(kBlk) void k_fc_bwd_weight(const float *dy, const float *x, float *dw, float *db, int B,
                                                       int In, int Out) {
    __shared__ float red[kBlk / 64][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t t = int64_t(blockIdx.x) * 64 + lane;
    const bool ok = t < int64_t(Out) * (In + 1);
    const int64_t tt = ok ? t : 0;
    const int i = int(tt % (In + 1));
    const int o = int(tt / (In + 1));
    float s = 0.0f;
    if (i < In) {
#pragma unroll 8
        for (int n = w; n < B; n += 4) s = fmaf(dy[int64_t(n) * Out + o], x[int64_t(n) * In + i], s);
    } else {
#pragma unroll 8
        for (int n = w; n < B; n += 4) s = fmaf(dy[int64_t(n) * Out + o], 1.0f, s);
    }
    red[w][lane] = s;
    __syncthreads();
    if (w != 0 || !ok) return;
    const float v = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    if (i < In)
        dw[int64_t(o) * In + i] = v;
    else
        db[o] = v;
}

// mean squared error: loss partials and dy = 2 (y - t) / (B * Out)
__global__ __launch_bounds__(kBlk) void k_mse(const float *y, const float *tgt, float *dy, float *loss_part,
                                             int64_t n, float scale) {
    __shared__ float red[kBlk];
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    float e = 0.0f;
    if (i < n) {
        const float d = y[i] - tgt[i];
        dy[i] = 2.0f * d * scale;
        e = d * d;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

__global__ void k_sum_loss(const float *part, int n, float scale, float *loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.0f;
        for (int i = 0; i < n; ++i) s += part[i];
        *loss = s * scale;
    }
}

// ----------------------------------------------------------------- Adam
__global__ __launch_bounds__(kBlk) void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 copies of a conv weight [Cout, 9, Cin]: forward layout and the
// flipped, transposed layout of the input-gradient product [Cin, 9, Cout].
// BF16 copies of the conv weights of layers 1..kLayers - 1 in one launch:
// wf in the [Cout][9][Cin] layout, wd flipped and transposed for the input
// gradient ([Cin][9][Cout], tap 8 - t).  Element i belongs to the layer
// whose range [start[l], start[l + 1]) holds it.
struct ConvWeights {
    const float *w[kLayers];
    u16 *wf[kLayers], *wd[kLayers];
    int cin[kLayers], cout[kLayers];
    int64_t start[kLayers + 1];
};

__global__ __launch_bounds__(kBlk) void k_conv_weights_bf16(ConvWeights cw) {
    const int64_t g = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (g >= cw.start[kLayers - 1]) return;
    int l = 0;
#pragma unroll
    for (int m = 1; m < kLayers - 1; ++m) l = g >= cw.start[m] ? m : l;
    const int64_t i = g - cw.start[l];
    const int Cin = cw.cin[l], Cout = cw.cout[l];
    const int ci = int(i % Cin);
    const int tap = int((i / Cin) % 9);
    const int co = int(i / (int64_t(9) * Cin));
    const u16 h = f2bf(cw.w[l][i]);
    cw.wf[l][i] = h;
    cw.wd[l][(int64_t(ci) * 9 + (8 - tap)) * Cout + co] = h;
}

// The full-resolution gradient from a pooled gradient and the masks (the
// test hook's view of a gradient that is not stored): one thread per
// full-resolution pixel and eight channels.
__global__ __launch_bounds__(kBlk) void k_expand_grad(const u16 *gp, const uint8_t *mask, u16 *out, int B, int H,
                                                     int W, int C) {
    const int64_t t = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (t >= int64_t(B) * H * W * (C / 8)) return;
    const int c8 = int(t % (C / 8));
    const int64_t p = t / (C / 8);
    const int x = int(p % W), y = int((p / W) % H);
    const int64_t n = p / (int64_t(H) * W);
    const int64_t e = ((n * (H / 2) + (y >> 1)) * (W / 2) + (x >> 1)) * C + 8 * c8;
    *reinterpret_cast<uint4 *>(out + p * C + 8 * c8) =
        expand8(*reinterpret_cast<const uint4 *>(gp + e), *reinterpret_cast<const uint2 *>(mask + e),
                ((y & 1) << 1) | (x & 1));
}

// Fixed-order sum of split partials for few outputs over many splits: one
// wavefront per output, lane l summing splits l, l + 64, ... in order, then
// a fixed butterfly over the lanes.
__global__ __launch_bounds__(kBlk) void k_sum_splits_wave(const float *partial, float *out, int64_t n, int splits) {
    const int64_t i = int64_t(blockIdx.x) * (kBlk / 64) + (threadIdx.x >> 6);
    if (i >= n) return;  // whole wavefronts
    const int lane = threadIdx.x & 63;
    float s = 0.0f;
    for (int k = lane; k < splits; k += 64) s += partial[int64_t(k) * n + i];
    s = wave_sum_f(s);
    if (lane == 0) out[i] = s;
}

// first-layer gradients: [co][10] sums (9 taps, then bias) -> weights, bias
__global__ __launch_bounds__(kBlk) void k_scatter_conv1(const float *sum, float *gw, float *gb, int C) {
    const int t = int(blockIdx.x) * kBlk + int(threadIdx.x);
    if (t >= C * 10) return;
    const int co = t / 10, k = t % 10;
    if (k < 9)
        gw[co * 9 + k] = sum[t];
    else
        gb[co] = sum[t];
}

inline unsigned nblk(int64_t n) { return unsigned((n + kBlk - 1) / kBlk); }

}  // namespace

// ======================================================================
// host side
// ======================================================================

struct lsm_cnn {
    lsm_cnn_config cfg{};
    int C[kLayers + 1];  // C[0] = 1 input channel
    int Hs[kLayers];     // spatial size of layer l's conv
    int64_t w_off[kLayers + 2], b_off[kLayers + 2], w_n[kLayers + 2];
    int64_t nparam = 0;
    bool bound = false;
    hipStream_t stream = nullptr;
    // device
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    u16 *wf[kLayers]{}, *wd[kLayers]{};
    // act: last conv output (post ReLU); pool: pooled outputs of the other
    // layers; mask: their ReLU masks (4 bits per pooled pixel and channel);
    // dact: conv output gradients; dpool: gradient of the first pooled map
    u16 *act = nullptr, *pool[kLayers]{}, *dact[kLayers]{}, *dpool0 = nullptr;
    // pooled gradient of layer 2's input (the full-resolution dact[1] is
    // then not stored: its consumers expand it with mask[1]); gp_used: the
    // last backward pass took that path
    u16 *gp = nullptr;
    bool gp_used = false;
    uint8_t *mask[kLayers]{};
    float *gap = nullptr, *h1 = nullptr, *y = nullptr;
    float *dgap = nullptr, *dh1 = nullptr, *dy = nullptr;
    float *part = nullptr;
    size_t part_n = 0;
    float *loss_part = nullptr, *loss = nullptr;
    const uint8_t *x_last = nullptr;
    int64_t b_last = 0;
    std::string err;
};

namespace {

// Allocation-free loss (lsm_cnn_mse_noalloc): the per-workgroup loss
// partials live in this file-scope device array, one copy per GPU, held
// until the process ends.  Host code never passes the array's name to a
// kernel (in host code it is only a stand-in for the symbol): the device
// address of each GPU's copy is looked up once per device, with that device
// current, and kept in scratch_ptr.
constexpr int kMseScratch = 65536;  // partials: batch x outputs <= 65536 x kBlk
__device__ __align__(256) float scratch[kMseScratch];
constexpr int kMaxDevices = 64;
float *scratch_ptr[kMaxDevices] = {};
std::mutex scratch_mu;

// Device address of this device's scratch array (nullptr on failure).
float *device_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        scratch_ptr[dev] = static_cast<float *>(ptr);
    }
    return scratch_ptr[dev];
}

int cfail(lsm_cnn *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define CHIP(c, call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return cfail((c), LSM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int64_t kSplitPix = 8192;  // pixels per weight-gradient split

int64_t splits_for(int64_t npix) { return (npix + kSplitPix - 1) / kSplitPix; }

// Weight-gradient splits of the layers with >= 32 input channels: about
// 512 workgroups over the (64 x 288) tiles, a multiple of 64 pixels each.
int64_t wgrad_pix_per_split(int64_t npix, int64_t cout, int64_t cin) {
    const int64_t tiles = ((cout + 63) / 64) * (9 * cin / kWwN);
    const int64_t sp = std::max<int64_t>(1, (512 + tiles - 1) / tiles);
    return std::max<int64_t>(64, ((npix + sp - 1) / sp + 63) / 64 * 64);
}

// The halo weight-gradient kernel: sides multiples of 8, whole 32-channel
// input blocks and 64-channel output blocks.  Splits are runs of 8 x 8
// tiles, about 512 workgroups in all.
bool wgrad_halo_ok(int64_t H, int64_t cin, int64_t cout) { return H % 8 == 0 && cin % 32 == 0 && cout % 64 == 0; }
int64_t wgrad_halo_tiles_per_split(int64_t ntiles, int64_t cout, int64_t cin) {
    const int64_t blocks = (cout / 64) * (cin / 32);
    const int64_t sp = std::max<int64_t>(1, (512 + blocks - 1) / blocks);
    return std::max<int64_t>(1, (ntiles + sp - 1) / sp);
}

size_t cnn_layout(const lsm_cnn *c, std::vector<size_t> *sizes) {
    const int64_t B = c->cfg.batch;
    const int64_t P = c->nparam;
    std::vector<size_t> s;
    s.push_back(P * 4);  // p
    s.push_back(P * 4);  // g
    s.push_back(P * 4);  // m
    s.push_back(P * 4);  // v
    for (int l = 1; l < kLayers; ++l) s.push_back(size_t(c->w_n[l]) * 2);  // wf
    for (int l = 1; l < kLayers; ++l) s.push_back(size_t(c->w_n[l]) * 2);  // wd
    // full-resolution conv outputs are stored only for the last layer; the
    // others are pooled in the conv epilogue and keep a ReLU mask
    const int L = kLayers - 1;
    s.push_back(size_t(B * c->Hs[L] * c->Hs[L] * c->C[L + 1]) * 2);  // act
    s.push_back(size_t(B * c->Hs[0] * c->Hs[0] / 4 * c->C[1]) * 2);  // dpool0
    s.push_back(size_t(B * c->Hs[2] * c->Hs[2] * c->C[2]) * 2);      // gp
    for (int l = 0; l < kLayers; ++l) {
        const int64_t hw = int64_t(c->Hs[l]) * c->Hs[l];
        s.push_back(l > 0 ? size_t(B * hw * c->C[l + 1]) * 2 : 0);       // dact
        s.push_back(l < L ? size_t(B * hw / 4 * c->C[l + 1]) * 2 : 0);   // pool
        // mask: 4 bits per pooled pixel and channel in the first layer, a byte in the others
        s.push_back(l > 0 && l < L ? size_t(B * hw / 4 * c->C[l + 1]) : (l == 0 ? size_t(B * hw / 4 * c->C[1] / 2) : 0));
    }
    const int hid = c->cfg.hidden, out = c->cfg.outputs;
    s.push_back(size_t(B) * c->C[kLayers] * 4);  // gap
    s.push_back(size_t(B) * c->C[kLayers] * 4);  // dgap
    s.push_back(size_t(B) * hid * 4);            // h1
    s.push_back(size_t(B) * hid * 4);            // dh1
    s.push_back(size_t(B) * out * 4);            // y
    s.push_back(size_t(B) * out * 4);            // dy
    s.push_back(c->part_n * 4);                  // split partials
    s.push_back(size_t(nblk(B * out)) * 4 + 256);  // loss partials + loss
    size_t o = 0;
    for (size_t x : s) o += al256(x);
    if (sizes) *sizes = s;
    return o;
}

}  // namespace

extern "C" {

int lsm_cnn_create(const lsm_cnn_config *cfg, lsm_cnn **out) {
    if (!cfg || !out) return LSM_EINVAL;
    *out = nullptr;
    const lsm_cnn_config &k = *cfg;
    if (k.batch < 1 || k.height < 16 || k.width < 16 || k.height % 16 || k.width % 16 || k.hidden < 1 ||
        k.outputs < 1)
        return LSM_EINVAL;
    for (int l = 0; l < kLayers; ++l)
        if (k.channels[l] != 32 && k.channels[l] != 64 && k.channels[l] != 128 && k.channels[l] != 256)
            return LSM_EINVAL;
    lsm_cnn *c = new (std::nothrow) lsm_cnn();
    if (!c) return LSM_ENOMEM;
    c->cfg = k;
    c->C[0] = 1;
    for (int l = 0; l < kLayers; ++l) c->C[l + 1] = k.channels[l];
    int h = k.height;
    for (int l = 0; l < kLayers; ++l) {
        c->Hs[l] = h;
        if (l < kLayers - 1) h /= 2;
    }
    if (k.width != k.height) {
        delete c;
        return LSM_EINVAL;  // square images
    }
    int64_t o = 0;
    for (int l = 0; l < kLayers; ++l) {
        c->w_off[l] = o;
        c->w_n[l] = int64_t(c->C[l + 1]) * 9 * c->C[l];
        o += c->w_n[l];
        c->b_off[l] = o;
        o += c->C[l + 1];
    }
    c->w_off[kLayers] = o;
    c->w_n[kLayers] = int64_t(k.hidden) * c->C[kLayers];
    o += c->w_n[kLayers];
    c->b_off[kLayers] = o;
    o += k.hidden;
    c->w_off[kLayers + 1] = o;
    c->w_n[kLayers + 1] = int64_t(k.outputs) * k.hidden;
    o += c->w_n[kLayers + 1];
    c->b_off[kLayers + 1] = o;
    o += k.outputs;
    c->nparam = o;
    // split partial buffer: max over layers of splits x (weights + bias)
    size_t pn = 0;
    for (int l = 0; l < kLayers; ++l) {
        const int64_t npix = int64_t(k.batch) * c->Hs[l] * c->Hs[l];
        const int64_t sp = splits_for(npix);
        pn = std::max(pn, size_t(sp * (c->w_n[l] + c->C[l + 1] * 10)));
        if (l > 0) {
            const int64_t pps = wgrad_pix_per_split(npix, c->C[l + 1], c->C[l]);
            const int64_t sw = (npix + pps - 1) / pps;
            pn = std::max(pn, size_t(sw * (c->w_n[l] + c->C[l + 1])));
            if (wgrad_halo_ok(c->Hs[l], c->C[l], c->C[l + 1])) {
                const int64_t nt = npix / 64, tps = wgrad_halo_tiles_per_split(nt, c->C[l + 1], c->C[l]);
                pn = std::max(pn, size_t((nt + tps - 1) / tps * (c->w_n[l] + c->C[l + 1])));
            }
        }
    }
    // slack for the first layer's summed [co][10] block after its partials
    c->part_n = pn + size_t(c->C[1]) * 10 + 64;
    *out = c;
    return LSM_OK;
}

void lsm_cnn_destroy(lsm_cnn *c) {
    if (!c) return;
    if (c->bound) (void)hipStreamSynchronize(c->stream);
    delete c;
}

const char *lsm_cnn_last_error(const lsm_cnn *c) { return c ? c->err.c_str() : "null network"; }

int lsm_cnn_param_count(const lsm_cnn *c, int64_t *n) {
    if (!c || !n) return LSM_EINVAL;
    *n = c->nparam;
    return LSM_OK;
}

int lsm_cnn_workspace_bytes(const lsm_cnn *c, size_t *bytes) {
    if (!c || !bytes) return LSM_EINVAL;
    *bytes = cnn_layout(c, nullptr);
    return LSM_OK;
}

int lsm_cnn_bind(lsm_cnn *c, void *dptr, size_t bytes, void *hip_stream) {
    if (!c || !dptr) return LSM_EINVAL;
    if (c->bound) return cfail(c, LSM_ESTATE, "already bound");
    if (reinterpret_cast<uintptr_t>(dptr) % 256) return cfail(c, LSM_EINVAL, "workspace must be 256-byte aligned");
    std::vector<size_t> s;
    const size_t need = cnn_layout(c, &s);
    if (bytes < need) return cfail(c, LSM_ENOMEM, "workspace too small");
    char *w = static_cast<char *>(dptr);
    size_t o = 0;
    size_t idx = 0;
    auto take = [&]() -> char * {
        char *r = w + o;
        o += al256(s[idx++]);
        return r;
    };
    c->p = reinterpret_cast<float *>(take());
    c->g = reinterpret_cast<float *>(take());
    c->m = reinterpret_cast<float *>(take());
    c->v = reinterpret_cast<float *>(take());
    for (int l = 1; l < kLayers; ++l) c->wf[l] = reinterpret_cast<u16 *>(take());
    for (int l = 1; l < kLayers; ++l) c->wd[l] = reinterpret_cast<u16 *>(take());
    c->act = reinterpret_cast<u16 *>(take());
    c->dpool0 = reinterpret_cast<u16 *>(take());
    c->gp = reinterpret_cast<u16 *>(take());
    for (int l = 0; l < kLayers; ++l) {
        c->dact[l] = reinterpret_cast<u16 *>(take());
        c->pool[l] = reinterpret_cast<u16 *>(take());
        c->mask[l] = reinterpret_cast<uint8_t *>(take());
    }
    c->gap = reinterpret_cast<float *>(take());
    c->dgap = reinterpret_cast<float *>(take());
    c->h1 = reinterpret_cast<float *>(take());
    c->dh1 = reinterpret_cast<float *>(take());
    c->y = reinterpret_cast<float *>(take());
    c->dy = reinterpret_cast<float *>(take());
    c->part = reinterpret_cast<float *>(take());
    c->loss_part = reinterpret_cast<float *>(take());
    c->loss = c->loss_part + nblk(int64_t(c->cfg.batch) * c->cfg.outputs);
    c->stream = static_cast<hipStream_t>(hip_stream);
    CHIP(c, hipMemsetAsync(w, 0, need, c->stream));
    CHIP(c, hipStreamSynchronize(c->stream));
    c->bound = true;
    return LSM_OK;
}

static int refresh_bf16(lsm_cnn *c) {
    ConvWeights cw{};
    cw.start[0] = 0;
    for (int l = 1; l < kLayers; ++l) {  // entry l - 1: conv layer l
        cw.w[l - 1] = c->p + c->w_off[l];
        cw.wf[l - 1] = c->wf[l];
        cw.wd[l - 1] = c->wd[l];
        cw.cin[l - 1] = c->C[l];
        cw.cout[l - 1] = c->C[l + 1];
        cw.start[l] = cw.start[l - 1] + c->w_n[l];
    }
    cw.start[kLayers] = cw.start[kLayers - 1];
    hipLaunchKernelGGL(k_conv_weights_bf16, dim3(nblk(cw.start[kLayers - 1])), dim3(kBlk), 0, c->stream, cw);
    CHIP(c, hipGetLastError());
    return LSM_OK;
}

int lsm_cnn_set_params(lsm_cnn *c, const float *host) {
    if (!c || !host) return LSM_EINVAL;
    if (!c->bound) return cfail(c, LSM_ESTATE, "bind first");
    CHIP(c, hipMemcpyAsync(c->p, host, size_t(c->nparam) * 4, hipMemcpyHostToDevice, c->stream));
    CHIP(c, hipMemsetAsync(c->m, 0, size_t(c->nparam) * 4, c->stream));
    CHIP(c, hipMemsetAsync(c->v, 0, size_t(c->nparam) * 4, c->stream));
    int rc = refresh_bf16(c);
    if (rc) return rc;
    CHIP(c, hipStreamSynchronize(c->stream));
    return LSM_OK;
}

static int get_vec(lsm_cnn *c, const float *src, float *host) {
    if (!c || !host) return LSM_EINVAL;
    if (!c->bound) return cfail(c, LSM_ESTATE, "bind first");
    CHIP(c, hipMemcpyAsync(host, src, size_t(c->nparam) * 4, hipMemcpyDeviceToHost, c->stream));
    CHIP(c, hipStreamSynchronize(c->stream));
    return LSM_OK;
}

int lsm_cnn_get_params(lsm_cnn *c, float *host) { return get_vec(c, c ? c->p : nullptr, host); }
int lsm_cnn_get_grads(lsm_cnn *c, float *host) { return get_vec(c, c ? c->g : nullptr, host); }

int lsm_cnn_forward(lsm_cnn *c, const uint8_t *x, int64_t batch, float *y) {
    if (!c || !x) return LSM_EINVAL;
    if (!c->bound) return cfail(c, LSM_ESTATE, "bind first");
    if (batch < 1 || batch > c->cfg.batch) return cfail(c, LSM_EINVAL, "batch out of range");
    const int B = int(batch);
    const int H0 = c->Hs[0];
    hipLaunchKernelGGL(k_conv1_pool_fwd, dim3(nblk(int64_t(B) * (H0 / 2) * (H0 / 2))), dim3(kBlk), 0, c->stream,
                       x, c->p + c->w_off[0], c->p + c->b_off[0], c->pool[0],
                       reinterpret_cast<uint32_t *>(c->mask[0]), B, H0, H0, c->C[1]);
    CHIP(c, hipGetLastError());
    for (int l = 1; l < kLayers; ++l) {
        const int H = c->Hs[l];
        const dim3 grid = conv_grid(int64_t(B) * H * H, c->C[l + 1]);
        const int tw = conv_lds_tw(H, H, c->C[l], c->C[l + 1]);
        const bool pool = l < kLayers - 1;
        if (tw && pool)
            launch_conv_lds<kEpiPool>(c->stream, tw, c->pool[l - 1], c->wf[l], c->p + c->b_off[l], c->pool[l],
                                      c->mask[l], B, H, c->C[l], c->C[l + 1]);
        else if (tw)
            launch_conv_lds<kEpiStore>(c->stream, tw, c->pool[l - 1], c->wf[l], c->p + c->b_off[l], c->act,
                                       nullptr, B, H, c->C[l], c->C[l + 1]);
        else if (pool)
            hipLaunchKernelGGL((k_conv_mfma<kEpiPool, kConvWM, kConvWN>), grid, dim3(kBlk), 0, c->stream,
                               c->pool[l - 1], c->wf[l], c->p + c->b_off[l], c->pool[l], nullptr, c->mask[l], B, H, H,
                               c->C[l], c->C[l + 1]);
        else
            hipLaunchKernelGGL((k_conv_mfma<kEpiStore, kConvWM, kConvWN>), grid, dim3(kBlk), 0, c->stream,
                               c->pool[l - 1], c->wf[l], c->p + c->b_off[l], c->act, nullptr, nullptr, B, H, H,
                               c->C[l], c->C[l + 1]);
        CHIP(c, hipGetLastError());
    }
    const int HL = c->Hs[kLayers - 1], CL = c->C[kLayers];
    hipLaunchKernelGGL(k_gap_fwd, dim3(nblk(int64_t(B) * CL)), dim3(kBlk), 0, c->stream, c->act, c->gap,
                       B, HL * HL, CL);
    const int hid = c->cfg.hidden, out = c->cfg.outputs;
    hipLaunchKernelGGL(k_fc_fwd, fc_grid(B, hid), dim3(kBlk), 0, c->stream, c->gap,
                       c->p + c->w_off[kLayers], c->p + c->b_off[kLayers], c->h1, B, CL, hid, 1);
    hipLaunchKernelGGL(k_fc_fwd, fc_grid(B, out), dim3(kBlk), 0, c->stream, c->h1,
                       c->p + c->w_off[kLayers + 1], c->p + c->b_off[kLayers + 1], c->y, B, hid, out, 0);
    CHIP(c, hipGetLastError());
    if (y) CHIP(c, hipMemcpyAsync(y, c->y, size_t(B) * out * 4, hipMemcpyDeviceToDevice, c->stream));
    c->x_last = x;
    c->b_last = B;
    return LSM_OK;
}

int lsm_cnn_mse(lsm_cnn *c, const float *target, float *dy, float *loss) {
    if (!c || !target) return LSM_EINVAL;
    if (!c->bound || c->b_last < 1) return cfail(c, LSM_ESTATE, "forward first");
    const int64_t n = c->b_last * c->cfg.outputs;
    const unsigned nb = nblk(n);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kBlk), 0, c->stream, c->y, target, c->dy, c->loss_part, n,
                       1.0f / float(n));
    hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(64), 0, c->stream, c->loss_part, int(nb), 1.0f / float(n), c->loss);
    CHIP(c, hipGetLastError());
    if (dy) CHIP(c, hipMemcpyAsync(dy, c->dy, size_t(n) * 4, hipMemcpyDeviceToDevice, c->stream));
    if (loss) CHIP(c, hipMemcpyAsync(loss, c->loss, 4, hipMemcpyDeviceToDevice, c->stream));
    return LSM_OK;
}

int lsm_cnn_mse_noalloc(lsm_cnn *c, const float *target, float *dy, float *loss) {
    if (!c || !target || !dy || !loss) return LSM_EINVAL;
    if (!c->bound || c->b_last < 1) return cfail(c, LSM_ESTATE, "forward first");
    const int64_t n = c->b_last * c->cfg.outputs;
    const int64_t nb = nblk(n);
    if (nb > kMseScratch)
        return cfail(c, LSM_EINVAL, "batch x outputs exceeds the allocation-free limit of " +
                                        std::to_string(int64_t(kMseScratch) * kBlk));
    int dev = 0;
    CHIP(c, hipGetDevice(&dev));
    float *part = device_scratch(dev);
    if (!part) return cfail(c, LSM_EHIP, "hipGetSymbolAddress of the scratch array failed");
    // the same kernels and summation order as lsm_cnn_mse; every partial the
    // sum reads is written first, so the array needs no clearing
    hipLaunchKernelGGL(k_mse, dim3(unsigned(nb)), dim3(kBlk), 0, c->stream, c->y, target, dy, part, n,
                       1.0f / float(n));
    hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(64), 0, c->stream, part, int(nb), 1.0f / float(n), loss);
    CHIP(c, hipGetLastError());
    return LSM_OK;
}

int lsm_cnn_backward(lsm_cnn *c, const float *dy) {
    if (!c) return LSM_EINVAL;
    if (!c->bound || c->b_last < 1) return cfail(c, LSM_ESTATE, "forward first");
    const int B = int(c->b_last);
    const int hid = c->cfg.hidden, out = c->cfg.outputs, CL = c->C[kLayers];
    if (dy && dy != c->dy) CHIP(c, hipMemcpyAsync(c->dy, dy, size_t(B) * out * 4, hipMemcpyDeviceToDevice, c->stream));
    // dense layers
    hipLaunchKernelGGL(k_fc_bwd_weight, dim3(unsigned((int64_t(out) * (hid + 1) + 63) / 64)), dim3(kBlk), 0, c->stream, c->dy, c->h1,
                       c->g + c->w_off[kLayers + 1], c->g + c->b_off[kLayers + 1], B, hid, out);
    hipLaunchKernelGGL(k_fc_bwd_data, dim3(nblk(int64_t(B) * hid)), dim3(kBlk), 0, c->stream, c->dy,
                       c->p + c->w_off[kLayers + 1], c->h1, c->dh1, B, hid, out);
    hipLaunchKernelGGL(k_fc_bwd_weight, dim3(unsigned((int64_t(hid) * (CL + 1) + 63) / 64)), dim3(kBlk), 0, c->stream, c->dh1, c->gap,
                       c->g + c->w_off[kLayers], c->g + c->b_off[kLayers], B, CL, hid);
    hipLaunchKernelGGL(k_fc_bwd_data, dim3(nblk(int64_t(B) * CL)), dim3(kBlk), 0, c->stream, c->dh1,
                       c->p + c->w_off[kLayers], nullptr, c->dgap, B, CL, hid);
    CHIP(c, hipGetLastError());
    const int HL = c->Hs[kLayers - 1];
    hipLaunchKernelGGL(k_gap_bwd_relu, dim3(nblk(int64_t(B) * HL * HL * (CL / 8))), dim3(kBlk), 0, c->stream, c->dgap,
                       c->act, c->dact[kLayers - 1], B, HL * HL, CL);
    CHIP(c, hipGetLastError());
    // The input gradient of layer 2 stays at its pooled resolution (gp) when
    // the kernels that consume the full-resolution one -- layer 1's halo
    // weight gradient and its 8 x 32-tile input gradient -- can expand it
    // with mask[1] themselves (the conditions of their launches below).
    const bool xin = c->C[3] == 128 && c->C[2] == 64 && c->Hs[2] % 16 == 0 &&
                     wgrad_halo_ok(c->Hs[1], c->C[1], c->C[2]) && c->C[1] % 32 == 0 && c->Hs[1] % 32 == 0;
    c->gp_used = xin;
    for (int l = kLayers - 1; l >= 0; --l) {
        const int H = c->Hs[l];
        const int64_t npix = int64_t(B) * H * H;
        const int64_t sp = splits_for(npix);
        const int64_t nw = c->w_n[l], cout = c->C[l + 1], cin = c->C[l];
        if (l > 0) {
            // weight gradient: MFMA over pixel splits, then a fixed-order sum
            int64_t sw;
            float *bias_part;
            if (wgrad_halo_ok(H, cin, cout)) {
                const int64_t nt = npix / 64, tps = wgrad_halo_tiles_per_split(nt, cout, cin);
                sw = (nt + tps - 1) / tps;
                bias_part = c->part + sw * nw;  // [split][co] after the weight partials
                const dim3 grid(unsigned(cout / 64), unsigned(cin / 32), unsigned(sw));
                if (l == 1 && xin)
                    hipLaunchKernelGGL(k_conv_wgrad_halo<true>, grid, dim3(kBlk), 0, c->stream, c->pool[l - 1], c->gp,
                                       c->mask[1], c->part, bias_part, B, H, H, int(cin), int(cout), int(tps));
                else
                    hipLaunchKernelGGL(k_conv_wgrad_halo<false>, grid, dim3(kBlk), 0, c->stream, c->pool[l - 1],
                                       c->dact[l], nullptr, c->part, bias_part, B, H, H, int(cin), int(cout),
                                       int(tps));
            } else {
                const int64_t pps = wgrad_pix_per_split(npix, cout, cin);
                sw = (npix + pps - 1) / pps;
                bias_part = c->part + sw * nw;
                const dim3 grid(unsigned((cout + 63) / 64), unsigned(9 * cin / kWwN), unsigned(sw));
                hipLaunchKernelGGL(k_conv_wgrad_wide, grid, dim3(kBlk), 0, c->stream, c->pool[l - 1], c->dact[l],
                                   c->part, bias_part, B, H, H, int(cin), int(cout), int(pps));
            }
            CHIP(c, hipGetLastError());
            hipLaunchKernelGGL(k_sum_splits, dim3(unsigned((nw + 63) / 64)), dim3(kBlk), 0, c->stream, c->part, c->g + c->w_off[l], nw,
                               int(sw));
            hipLaunchKernelGGL(k_sum_splits_wave, dim3(unsigned((cout + kBlk / 64 - 1) / (kBlk / 64))), dim3(kBlk), 0,
                               c->stream, bias_part, c->g + c->b_off[l], cout, int(sw));
            CHIP(c, hipGetLastError());
            // input gradient: implicit GEMM with the flipped weights; its
            // epilogue applies the pooling and ReLU of the layer below (the
            // first layer's backward takes the pooled gradient itself)
            const dim3 g2 = conv_grid(npix, int(cin));
            const dim3 g16(unsigned(B * (H / 8) * (H / 16)), 1);
            if (l == 2 && xin)
                // the pooled gradient of layer 2's input, kept at its own resolution
                hipLaunchKernelGGL((k_conv_lds128<16, 64, kEpiRaw, 8>), g16, dim3(kBlk), 0, c->stream, c->dact[l],
                                   c->wd[l], nullptr, c->gp, nullptr, B, H, H, int(cin));
            else if (l > 1 && cout == 128 && cin == 64 && H % 16 == 0)
                // staged-patch kernel (same K order, same bits); the mask
                // slot carries the masks of the layer below, read
                hipLaunchKernelGGL((k_conv_lds128<16, 64, kEpiExpand, 8>), g16, dim3(kBlk), 0, c->stream, c->dact[l],
                                   c->wd[l], nullptr, c->dact[l - 1], c->mask[l - 1], B, H, H, int(cin));
            else if (l > 1 && cout == 128 && cin == 128 && H % 16 == 0)
                hipLaunchKernelGGL((k_conv_lds128<16, 128, kEpiExpand, 8>), g16, dim3(kBlk), 0, c->stream, c->dact[l],
                                   c->wd[l], nullptr, c->dact[l - 1], c->mask[l - 1], B, H, H, int(cin));
            else if (l > 1 && cout == 256 && cin % 128 == 0 && H % 8 == 0)
                hipLaunchKernelGGL((k_conv_lds256<8, 128, kEpiExpand>), dim3(unsigned(B * (H / 8) * (H / 8)),
                                   unsigned(cin / 128)), dim3(kBlk), 0, c->stream, c->dact[l], c->wd[l], nullptr,
                                   c->dact[l - 1], c->mask[l - 1], B, H, H, int(cin));
            else if (l > 1)
                hipLaunchKernelGGL((k_conv_mfma<kEpiExpand, kConvWM, kConvWN>), g2, dim3(kBlk), 0, c->stream,
                                   c->dact[l], c->wd[l], nullptr, c->dact[l - 1], c->mask[l - 1], nullptr, B, H, H,
                                   int(cout), int(cin));
            else if (xin)
                // (l == 1) the same kernel expanding the pooled gradient while staging
                hipLaunchKernelGGL((k_conv_lds<64, 32, 32, kEpiRaw, 8, true>), dim3(unsigned(B * (H / 8) * (H / 32)),
                                   unsigned(cin / 32)), dim3(kBlk), 0, c->stream, c->gp, c->wd[l], nullptr,
                                   c->dpool0, nullptr, B, H, H, int(cin), c->mask[1]);
            else if (cout == 64 && cin % 32 == 0 && H % 32 == 0)
                // the staged-patch kernel (same K order, same bits): 64-channel
                // gradient input, 32-channel blocks of the output, 8 x 32 tiles
                // (two wavefronts of 128 pixels per 16 channels)
                hipLaunchKernelGGL((k_conv_lds<64, 32, 32, kEpiRaw, 8>), dim3(unsigned(B * (H / 8) * (H / 32)),
                                   unsigned(cin / 32)), dim3(kBlk), 0, c->stream, c->dact[l], c->wd[l], nullptr,
                                   c->dpool0, nullptr, B, H, H, int(cin));
            else if (cout == 64 && cin % 32 == 0 && H % 16 == 0)
                hipLaunchKernelGGL((k_conv_lds<64, 16, 32, kEpiRaw, 4>), dim3(unsigned(B * (H / 8) * (H / 16)),
                                   unsigned(cin / 32)), dim3(kBlk), 0, c->stream, c->dact[l], c->wd[l], nullptr,
                                   c->dpool0, nullptr, B, H, H, int(cin));
            else
                hipLaunchKernelGGL((k_conv_mfma<kEpiRaw, kConvWM, kConvWN>), g2, dim3(kBlk), 0, c->stream,
                                   c->dact[l], c->wd[l], nullptr, c->dpool0, nullptr, nullptr, B, H, H, int(cout),
                                   int(cin));
            CHIP(c, hipGetLastError());
        } else {
            const unsigned groups = unsigned((cout / kC1Cpw + kBlk / 64 - 1) / (kBlk / 64));
            if ((H / 2) % 64 == 0 && (H / 2) % kC1Rows == 0 && kC1Rows * 64 == kSplitPix / 4)
                // (row blocks x column chunks = the sp splits of kSplitPix / 4 pooled pixels)
                hipLaunchKernelGGL(k_conv1_bwd_rows, dim3(unsigned(sp), groups), dim3(kBlk), 0, c->stream, c->x_last,
                                   reinterpret_cast<const uint32_t *>(c->mask[0]), c->dpool0, c->part, B, H, H,
                                   int(cout));
            else
                hipLaunchKernelGGL(k_conv1_bwd, dim3(unsigned(sp), groups), dim3(kBlk), 0, c->stream, c->x_last,
                                   reinterpret_cast<const uint32_t *>(c->mask[0]), c->dpool0, c->part, B, H, H,
                                   int(cout), int64_t(kSplitPix / 4));
            // part layout [split][co][10]: taps then bias
            hipLaunchKernelGGL(k_sum_splits_wave, dim3(unsigned((cout * 10 + kBlk / 64 - 1) / (kBlk / 64))),
                               dim3(kBlk), 0, c->stream, c->part, c->part + sp * cout * 10, cout * 10, int(sp));
            CHIP(c, hipGetLastError());
            hipLaunchKernelGGL(k_scatter_conv1, dim3(nblk(cout * 10)), dim3(kBlk), 0, c->stream,
                               c->part + sp * cout * 10, c->g + c->w_off[0], c->g + c->b_off[0], int(cout));
            CHIP(c, hipGetLastError());
        }
    }
    return LSM_OK;
}

int lsm_cnn_adam_step(lsm_cnn *c, float lr, float beta1, float beta2, float eps, int64_t t) {
    if (!c || t < 1) return LSM_EINVAL;
    if (!c->bound) return cfail(c, LSM_ESTATE, "bind first");
    const float c1 = 1.0f - std::pow(beta1, float(t)), c2 = 1.0f - std::pow(beta2, float(t));
    hipLaunchKernelGGL(k_adam, dim3(nblk(c->nparam)), dim3(kBlk), 0, c->stream, c->p, c->g, c->m, c->v, c->nparam, lr,
                       beta1, beta2, eps, c1, c2);
    CHIP(c, hipGetLastError());
    return refresh_bf16(c);
}

int lsm_cnn_layout(const lsm_cnn *c, int64_t *w_off, int64_t *b_off, int64_t *w_n) {
    if (!c) return LSM_EINVAL;
    for (int l = 0; l < kLayers + 2; ++l) {
        if (w_off) w_off[l] = c->w_off[l];
        if (b_off) b_off[l] = c->b_off[l];
        if (w_n) w_n[l] = c->w_n[l];
    }
    return LSM_OK;
}

int lsm_cnn_read_buffer(lsm_cnn *c, int buffer, int layer, void *host, size_t *bytes) {
    if (!c || !bytes) return LSM_EINVAL;
    if (!c->bound) return cfail(c, LSM_ESTATE, "bind first");
    const int64_t B = c->cfg.batch;
    const int L = kLayers - 1;
    const void *src = nullptr;
    size_t n = 0;
    const bool lok = layer >= 0 && layer < kLayers;
    const int64_t hw = lok ? int64_t(c->Hs[layer]) * c->Hs[layer] : 0;
    const int64_t ch = lok ? c->C[layer + 1] : 0;
    switch (buffer) {
    case LSM_CNN_BUF_POOLED:
        if (lok && layer < L) src = c->pool[layer], n = size_t(B * hw / 4 * ch) * 2;
        break;
    case LSM_CNN_BUF_MASK:
        if (lok && layer > 0 && layer < L) src = c->mask[layer], n = size_t(B * hw / 4 * ch);
        break;
    case LSM_CNN_BUF_ACT:
        src = c->act, n = size_t(B * c->Hs[L] * c->Hs[L] * c->C[L + 1]) * 2;
        break;
    case LSM_CNN_BUF_DACT:
        if (lok && layer > 0) src = c->dact[layer], n = size_t(B * hw * ch) * 2;
        if (lok && layer == 1 && c->gp_used && host) {
            // not stored by the backward pass: expand the pooled gradient
            hipLaunchKernelGGL(k_expand_grad, dim3(nblk(int64_t(B) * hw * (ch / 8))), dim3(kBlk), 0, c->stream,
                               c->gp, c->mask[1], c->dact[1], int(B), c->Hs[1], c->Hs[1], int(ch));
            CHIP(c, hipGetLastError());
        }
        break;
    case LSM_CNN_BUF_DPOOL0:
        src = c->dpool0, n = size_t(B * c->Hs[0] * c->Hs[0] / 4 * c->C[1]) * 2;
        break;
    case LSM_CNN_BUF_GAP: src = c->gap, n = size_t(B) * c->C[kLayers] * 4; break;
    case LSM_CNN_BUF_DGAP: src = c->dgap, n = size_t(B) * c->C[kLayers] * 4; break;
    case LSM_CNN_BUF_HIDDEN: src = c->h1, n = size_t(B) * c->cfg.hidden * 4; break;
    case LSM_CNN_BUF_DHIDDEN: src = c->dh1, n = size_t(B) * c->cfg.hidden * 4; break;
    case LSM_CNN_BUF_OUT: src = c->y, n = size_t(B) * c->cfg.outputs * 4; break;
    case LSM_CNN_BUF_DOUT: src = c->dy, n = size_t(B) * c->cfg.outputs * 4; break;
    default: break;
    }
    if (!src) return cfail(c, LSM_EINVAL, "no such buffer");
    if (!host) {
        *bytes = n;
        return LSM_OK;
    }
    if (*bytes < n) return cfail(c, LSM_ENOMEM, "host buffer too small");
    CHIP(c, hipMemcpyAsync(host, src, n, hipMemcpyDeviceToHost, c->stream));
    CHIP(c, hipStreamSynchronize(c->stream));
    *bytes = n;
    return LSM_OK;
}

int lsm_cnn_conv_forward(lsm_cnn *c, int layer, const void *in, void *out, int64_t batch) {
    // single layer of the implicit-GEMM convolution (layers 1..4) on caller
    // buffers, with this network's weights: used to test the kernel alone
    if (!c || !in || !out || layer < 1 || layer >= kLayers || batch < 1) return LSM_EINVAL;
    if (!c->bound) return cfail(c, LSM_ESTATE, "bind first");
    const int H = c->Hs[layer];
    const int64_t npix = batch * H * H;
    hipLaunchKernelGGL((k_conv_mfma<kEpiStore, kConvWM, kConvWN>), conv_grid(npix, c->C[layer + 1]), dim3(kBlk), 0,
                       c->stream, static_cast<const u16 *>(in), c->wf[layer], c->p + c->b_off[layer],
                       static_cast<u16 *>(out), nullptr, nullptr, int(batch), H, H, c->C[layer], c->C[layer + 1]);
    CHIP(c, hipGetLastError());
    return LSM_OK;
}

}  // extern "C"
