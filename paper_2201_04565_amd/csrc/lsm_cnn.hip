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
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
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
    // round to nearest even (inputs are finite)
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u16(u >> 16);
}
__device__ inline float bf2f(u16 h) { return __uint_as_float(unsigned(h) << 16); }

union Frag {
    uint4 u;
    bf16x8 v;
};

// ------------------------------------------------------------------ conv 1
// One input channel (the phase image, uint8 0/1): direct FP32 convolution,
// each thread one output pixel x all output channels, ReLU, BF16 out.
__global__ __launch_bounds__(kBlk) void k_conv1_fwd(const uint8_t *x, const float *w, const float *b,
                                                   u16 *out, int B, int H, int W, int C) {
    const int64_t p = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (p >= int64_t(B) * H * W) return;
    const int xx = int(p % W), yy = int((p / W) % H);
    const int64_t n = p / (int64_t(H) * W);
    float v[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int sy = yy + t / 3 - 1, sx = xx + t % 3 - 1;
        v[t] = (sy >= 0 && sy < H && sx >= 0 && sx < W) ? float(x[(n * H + sy) * W + sx]) : 0.0f;
    }
    // eight channels per 16-byte store (C is a multiple of 32)
    for (int c0 = 0; c0 < C; c0 += 8) {
        u16 h[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float s = b[c0 + e];
#pragma unroll
            for (int t = 0; t < 9; ++t) s = fmaf(w[(c0 + e) * 9 + t], v[t], s);
            h[e] = f2bf(fmaxf(s, 0.0f));
        }
        *reinterpret_cast<uint4 *>(out + p * C + c0) = *reinterpret_cast<const uint4 *>(h);
    }
}

// ------------------------------------------------------ implicit-GEMM conv
// out[p, co] = act(sum_{tap, ci} in[shift(p, tap), ci] * wt[co, tap, ci] + bias[co])
// in: [B, H, W, Cin] BF16, wt: [Cout, 9, Cin] BF16, out: [B, H, W, Cout] BF16.
// Each wavefront owns WM x WN MFMA tiles of 16 x 16 (WM * 16 pixels x WN *
// 16 channels); the four wavefronts of a workgroup stack along pixels.  Per
// K step of 32 a lane issues WM + WN 16-byte loads for WM * WN MFMAs.
template <bool BIAS_RELU, int WM, int WN>
__global__ __launch_bounds__(kBlk) void k_conv_mfma(const u16 *in, const u16 *wt, const float *bias,
                                                   u16 *out, int B, int H, int W, int Cin, int Cout) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t npix = int64_t(B) * H * W;
    const int64_t p0 = (int64_t(blockIdx.x) * 4 + wv) * (WM * 16);
    const int c0 = blockIdx.y * (WN * 16);
    const int r16 = lane & 15, kq = lane >> 4;  // row within the 16-tile, K quarter
    int py[WM], px[WM];
    int64_t pn[WM];
    bool pok[WM];
#pragma unroll
    for (int r = 0; r < WM; ++r) {
        const int64_t p = p0 + r * 16 + r16;
        pok[r] = p < npix;
        const int64_t pp = pok[r] ? p : 0;
        px[r] = int(pp % W);
        py[r] = int((pp / W) % H);
        pn[r] = pp / (int64_t(H) * W);
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
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const u16 *arow[WM];
        bool aok[WM];
#pragma unroll
        for (int r = 0; r < WM; ++r) {
            const int sy = py[r] + dy, sx = px[r] + dx;
            aok[r] = pok[r] && sy >= 0 && sy < H && sx >= 0 && sx < W;
            arow[r] = in + (aok[r] ? ((pn[r] * H + sy) * W + sx) * Cin : 0) + 8 * kq;
        }
        for (int ci0 = 0; ci0 < Cin; ci0 += 32) {
            Frag a[WM], bfr[WN];
#pragma unroll
            for (int r = 0; r < WM; ++r) {
                const uint4 t = *reinterpret_cast<const uint4 *>(arow[r] + ci0);
                a[r].u = aok[r] ? t : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int c = 0; c < WN; ++c) {
                const uint4 t = *reinterpret_cast<const uint4 *>(wrow[c] + tap * Cin + ci0);
                bfr[c].u = cok[c] ? t : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < WM; ++r)
#pragma unroll
                for (int c = 0; c < WN; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r].v, bfr[c].v, acc[r][c], 0, 0, 0);
        }
    }
    // D layout: lane holds rows 4 * kq + i (pixels), column r16 (channel)
#pragma unroll
    for (int r = 0; r < WM; ++r)
#pragma unroll
        for (int c = 0; c < WN; ++c) {
            const int co = c0 + c * 16 + r16;
            if (co >= Cout) continue;
            const float bv = BIAS_RELU ? bias[co] : 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t p = p0 + r * 16 + 4 * kq + i;
                if (p >= npix) continue;
                float v = acc[r][c][i] + bv;
                if (BIAS_RELU) v = fmaxf(v, 0.0f);
                out[p * Cout + co] = f2bf(v);
            }
        }
}

constexpr int kConvWM = 4, kConvWN = 4;  // 64 pixels x 64 channels per wavefront

// ------------------------------------------------------- weight gradient
// dw[co, tap, ci] = sum_p dout[p, co] * in[shift(p, tap), ci], split over
// pixel ranges: partial[split][co][tap][ci] (FP32).  Workgroup tile: 64 co x
// 64 ci for one tap; K = 64 pixels per LDS stage.
__global__ __launch_bounds__(kBlk) void k_conv_wgrad_mfma(const u16 *in, const u16 *dout, float *partial,
                                                         int B, int H, int W, int Cin, int Cout,
                                                         int64_t pix_per_split) {
    __shared__ u16 sd[64][64 + 8];  // [co][pixel]
    __shared__ u16 sx[64][64 + 8];  // [ci][pixel]
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int co_t = blockIdx.x * 64, ci_t = (blockIdx.y % ((Cin + 63) / 64)) * 64;
    const int tap = blockIdx.y / ((Cin + 63) / 64);
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int split = blockIdx.z;
    const int64_t npix = int64_t(B) * H * W;
    const int64_t pbeg = int64_t(split) * pix_per_split;
    const int64_t pend = pbeg + pix_per_split < npix ? pbeg + pix_per_split : npix;
    const int r16 = lane & 15, kq = lane >> 4;
    const int wco = (wv >> 1) * 32, wci = (wv & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    // loader: thread t covers pixel t / 4, channels (t % 4) * 16 .. + 15
    const int lp = threadIdx.x >> 2, lc = (threadIdx.x & 3) * 16;
    for (int64_t q0 = pbeg; q0 < pend; q0 += 64) {
        const int64_t p = q0 + lp;
        const bool pin = p < pend;
        const int64_t pp = pin ? p : 0;
        const int x = int(pp % W), y = int((pp / W) % H);
        const int64_t n = pp / (int64_t(H) * W);
        const int sy = y + dy, sx2 = x + dx;
        const bool xin = pin && sy >= 0 && sy < H && sx2 >= 0 && sx2 < W;
        const int64_t xb = xin ? ((n * H + sy) * W + sx2) * Cin : 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int cc = lc + 8 * h;
            uint4 vd = make_uint4(0, 0, 0, 0), vx = make_uint4(0, 0, 0, 0);
            if (pin && co_t + cc < Cout) vd = *reinterpret_cast<const uint4 *>(dout + pp * Cout + co_t + cc);
            if (xin && ci_t + cc < Cin) vx = *reinterpret_cast<const uint4 *>(in + xb + ci_t + cc);
            const u16 *ed = reinterpret_cast<const u16 *>(&vd);
            const u16 *ex = reinterpret_cast<const u16 *>(&vx);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                sd[cc + e][lp] = ed[e];
                sx[cc + e][lp] = ex[e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            Frag a[2], b[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) a[r].u = *reinterpret_cast<const uint4 *>(&sd[wco + r * 16 + r16][ks * 32 + 8 * kq]);
#pragma unroll
            for (int c = 0; c < 2; ++c) b[c].u = *reinterpret_cast<const uint4 *>(&sx[wci + c * 16 + r16][ks * 32 + 8 * kq]);
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r].v, b[c].v, acc[r][c], 0, 0, 0);
        }
        __syncthreads();
    }
    // D: rows = co (4 * kq + i), column = ci (r16)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int ci = ci_t + wci + c * 16 + r16;
            if (ci >= Cin) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = co_t + wco + r * 16 + 4 * kq + i;
                if (co >= Cout) continue;
                partial[((int64_t(split) * Cout + co) * 9 + tap) * Cin + ci] = acc[r][c][i];
            }
        }
}

// Fixed-order sum of split partials (and bias gradient partials).
__global__ __launch_bounds__(kBlk) void k_sum_splits(const float *partial, float *out, int64_t n, int splits) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int k = 0; k < splits; ++k) s += partial[int64_t(k) * n + i];
    out[i] = s;
}

// db[c] partials: column sums of a [npix, C] BF16 matrix over pixel chunks.
// Thread t reads channel t % C of pixels t / C, t / C + 256 / C, ... (rows
// are contiguous, so a wavefront reads whole rows); the 256 / C partial sums
// of a channel are then added in a fixed order.
__global__ __launch_bounds__(kBlk) void k_colsum_bf16(const u16 *g, float *partial, int64_t npix, int C,
                                                     int64_t pix_per_split) {
    __shared__ float red[kBlk];
    const int c = threadIdx.x % C;
    const int lanes = kBlk / C;  // pixels read per pass (C divides 256)
    const int sub = threadIdx.x / C;
    const int64_t b0 = int64_t(blockIdx.x) * pix_per_split;
    const int64_t b1 = b0 + pix_per_split < npix ? b0 + pix_per_split : npix;
    float s = 0.0f;
    if (sub < lanes)
        for (int64_t p = b0 + sub; p < b1; p += lanes) s += bf2f(g[p * C + c]);
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < C) {
        float t = 0.0f;
        for (int k = 0; k < lanes; ++k) t += red[k * C + threadIdx.x];
        partial[int64_t(blockIdx.x) * C + threadIdx.x] = t;
    }
}

// Weight gradient of the one-channel first layer: partials [split][co][10]
// (9 taps, then the bias).  Wavefront w of a workgroup handles channels
// 8 w .. 8 w + 7 (workgroups along y cover further groups); its 64 lanes
// stride over the split's pixels and the lane sums are combined by a fixed
// wavefront reduction.
__device__ inline float wave_sum_f(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__global__ __launch_bounds__(kBlk) void k_conv1_wgrad(const uint8_t *x, const u16 *dout, float *partial, int B,
                                                     int H, int W, int C, int64_t pix_per_split) {
    const int lane = threadIdx.x & 63;
    const int grp = (blockIdx.y * (kBlk / 64)) + (threadIdx.x >> 6);
    if (grp * 8 >= C) return;  // whole wavefronts leave together
    const int64_t npix = int64_t(B) * H * W;
    const int64_t b0 = int64_t(blockIdx.x) * pix_per_split;
    const int64_t b1 = b0 + pix_per_split < npix ? b0 + pix_per_split : npix;
    float acc[8][10];
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int k = 0; k < 10; ++k) acc[e][k] = 0.0f;
    for (int64_t p = b0 + lane; p < b1; p += 64) {
        const uint4 gv = *reinterpret_cast<const uint4 *>(dout + p * C + grp * 8);
        const u16 *gh = reinterpret_cast<const u16 *>(&gv);
        const int xx = int(p % W), yy = int((p / W) % H);
        const int64_t n = p / (int64_t(H) * W);
        float v[10];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int sy = yy + t / 3 - 1, sx = xx + t % 3 - 1;
            v[t] = (sy >= 0 && sy < H && sx >= 0 && sx < W) ? float(x[(n * H + sy) * W + sx]) : 0.0f;
        }
        v[9] = 1.0f;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float g = bf2f(gh[e]);
#pragma unroll
            for (int k = 0; k < 10; ++k) acc[e][k] = fmaf(g, v[k], acc[e][k]);
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const float t = wave_sum_f(acc[e][k]);
            if (lane == 0) partial[(int64_t(blockIdx.x) * C + grp * 8 + e) * 10 + k] = t;
        }
}

// ------------------------------------------------------ pooling and GAP
__global__ __launch_bounds__(kBlk) void k_pool2_fwd(const u16 *in, u16 *out, int B, int H, int W, int C) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2;
    if (i >= int64_t(B) * Ho * Wo * C) return;
    const int c = int(i % C);
    const int64_t q = i / C;
    const int xo = int(q % Wo), yo = int((q / Wo) % Ho);
    const int64_t n = q / (int64_t(Ho) * Wo);
    float s = 0.0f;
#pragma unroll
    for (int d = 0; d < 4; ++d) s += bf2f(in[((n * H + 2 * yo + d / 2) * W + 2 * xo + d % 2) * C + c]);
    out[i] = f2bf(0.25f * s);
}

// gradient of pooling, times the ReLU mask of the pooled layer's output
__global__ __launch_bounds__(kBlk) void k_pool2_bwd_relu(const u16 *dpool, const u16 *act, u16 *dact, int B, int H,
                                                        int W, int C) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (i >= int64_t(B) * H * W * C) return;
    const int c = int(i % C);
    const int64_t q = i / C;
    const int x = int(q % W), y = int((q / W) % H);
    const int64_t n = q / (int64_t(H) * W);
    const float g = 0.25f * bf2f(dpool[((n * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c]);
    dact[i] = f2bf(bf2f(act[i]) > 0.0f ? g : 0.0f);
}

// ReLU mask applied to an input gradient in place
__global__ __launch_bounds__(kBlk) void k_relu_mask(u16 *g, const u16 *act, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (i >= n) return;
    if (!(bf2f(act[i]) > 0.0f)) g[i] = 0;
}

__global__ __launch_bounds__(kBlk) void k_gap_fwd(const u16 *in, float *out, int B, int HW, int C) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (i >= int64_t(B) * C) return;
    const int c = int(i % C);
    const int64_t n = i / C;
    float s = 0.0f;
    for (int p = 0; p < HW; ++p) s += bf2f(in[(n * HW + p) * C + c]);
    out[i] = s / float(HW);
}

__global__ __launch_bounds__(kBlk) void k_gap_bwd_relu(const float *dg, const u16 *act, u16 *dact, int B, int HW,
                                                      int C) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (i >= int64_t(B) * HW * C) return;
    const int c = int(i % C);
    const int64_t n = i / (int64_t(HW) * C);
    const float g = dg[n * C + c] / float(HW);
    dact[i] = f2bf(bf2f(act[i]) > 0.0f ? g : 0.0f);
}

// ---------------------------------------------------------- dense layers
// y[n, o] = act(b[o] + sum_i w[o, i] x[n, i])
__global__ __launch_bounds__(kBlk) void k_fc_fwd(const float *x, const float *w, const float *b, float *y, int B,
                                                int In, int Out, int relu) {
    const int64_t t = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (t >= int64_t(B) * Out) return;
    const int o = int(t % Out);
    const int64_t n = t / Out;
    float s = b[o];
    for (int i = 0; i < In; ++i) s = fmaf(w[int64_t(o) * In + i], x[n * In + i], s);
    y[t] = relu ? fmaxf(s, 0.0f) : s;
}

// dx[n, i] = sum_o w[o, i] dy[n, o], times the ReLU mask of x when given
__global__ __launch_bounds__(kBlk) void k_fc_bwd_data(const float *dy, const float *w, const float *xact,
                                                     float *dx, int B, int In, int Out) {
    const int64_t t = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (t >= int64_t(B) * In) return;
    const int i = int(t % In);
    const int64_t n = t / In;
    float s = 0.0f;
    for (int o = 0; o < Out; ++o) s = fmaf(w[int64_t(o) * In + i], dy[n * Out + o], s);
    if (xact && !(xact[t] > 0.0f)) s = 0.0f;
    dx[t] = s;
}

// dw[o, i] = sum_n dy[n, o] x[n, i]; db[o] = sum_n dy[n, o] (column In)
__global__ __launch_bounds__(kBlk) void k_fc_bwd_weight(const float *dy, const float *x, float *dw, float *db, int B,
                                                       int In, int Out) {
    const int64_t t = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (t >= int64_t(Out) * (In + 1)) return;
    const int i = int(t % (In + 1));
    const int o = int(t / (In + 1));
    float s = 0.0f;
    for (int n = 0; n < B; ++n) s = fmaf(dy[int64_t(n) * Out + o], i < In ? x[int64_t(n) * In + i] : 1.0f, s);
    if (i < In)
        dw[int64_t(o) * In + i] = s;
    else
        db[o] = s;
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
__global__ __launch_bounds__(kBlk) void k_conv_weights_bf16(const float *w, u16 *wf, u16 *wd, int Cin, int Cout) {
    const int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x;
    if (i >= int64_t(Cout) * 9 * Cin) return;
    const int ci = int(i % Cin);
    const int tap = int((i / Cin) % 9);
    const int co = int(i / (int64_t(9) * Cin));
    const u16 h = f2bf(w[i]);
    wf[i] = h;
    if (wd) wd[(int64_t(ci) * 9 + (8 - tap)) * Cout + co] = h;
}

// first-layer gradients: [co][10] sums (9 taps, then bias) -> weights, bias
__global__ void k_scatter_conv1(const float *sum, float *gw, float *gb, int C) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
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
    u16 *act[kLayers]{}, *pool[kLayers]{};    // conv outputs (post ReLU) and pooled
    u16 *dact[kLayers]{}, *dpool[kLayers]{};  // their gradients
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
    for (int l = 0; l < kLayers; ++l) {
        const int64_t hw = int64_t(c->Hs[l]) * c->Hs[l];
        s.push_back(size_t(B * hw * c->C[l + 1]) * 2);  // act
        s.push_back(size_t(B * hw * c->C[l + 1]) * 2);  // dact
        s.push_back(size_t(B * hw / 4 * c->C[l + 1]) * 2);  // pool
        s.push_back(size_t(B * hw / 4 * c->C[l + 1]) * 2);  // dpool
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
    for (int l = 0; l < kLayers; ++l) {
        c->act[l] = reinterpret_cast<u16 *>(take());
        c->dact[l] = reinterpret_cast<u16 *>(take());
        c->pool[l] = reinterpret_cast<u16 *>(take());
        c->dpool[l] = reinterpret_cast<u16 *>(take());
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
    for (int l = 1; l < kLayers; ++l) {
        hipLaunchKernelGGL(k_conv_weights_bf16, dim3(nblk(c->w_n[l])), dim3(kBlk), 0, c->stream,
                           c->p + c->w_off[l], c->wf[l], c->wd[l], c->C[l], c->C[l + 1]);
        CHIP(c, hipGetLastError());
    }
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
    hipLaunchKernelGGL(k_conv1_fwd, dim3(nblk(int64_t(B) * H0 * H0)), dim3(kBlk), 0, c->stream, x,
                       c->p + c->w_off[0], c->p + c->b_off[0], c->act[0], B, H0, H0, c->C[1]);
    CHIP(c, hipGetLastError());
    for (int l = 0; l < kLayers; ++l) {
        const int H = c->Hs[l];
        if (l > 0) {
            const int64_t npix = int64_t(B) * H * H;
            const dim3 grid(unsigned((npix + 64 * kConvWM - 1) / (64 * kConvWM)),
                            unsigned((c->C[l + 1] + 16 * kConvWN - 1) / (16 * kConvWN)));
            hipLaunchKernelGGL((k_conv_mfma<true, kConvWM, kConvWN>), grid, dim3(kBlk), 0, c->stream, c->pool[l - 1], c->wf[l],
                               c->p + c->b_off[l], c->act[l], B, H, H, c->C[l], c->C[l + 1]);
            CHIP(c, hipGetLastError());
        }
        if (l < kLayers - 1) {
            hipLaunchKernelGGL(k_pool2_fwd, dim3(nblk(int64_t(B) * (H / 2) * (H / 2) * c->C[l + 1])), dim3(kBlk), 0,
                               c->stream, c->act[l], c->pool[l], B, H, H, c->C[l + 1]);
            CHIP(c, hipGetLastError());
        }
    }
    const int HL = c->Hs[kLayers - 1], CL = c->C[kLayers];
    hipLaunchKernelGGL(k_gap_fwd, dim3(nblk(int64_t(B) * CL)), dim3(kBlk), 0, c->stream, c->act[kLayers - 1], c->gap,
                       B, HL * HL, CL);
    const int hid = c->cfg.hidden, out = c->cfg.outputs;
    hipLaunchKernelGGL(k_fc_fwd, dim3(nblk(int64_t(B) * hid)), dim3(kBlk), 0, c->stream, c->gap,
                       c->p + c->w_off[kLayers], c->p + c->b_off[kLayers], c->h1, B, CL, hid, 1);
    hipLaunchKernelGGL(k_fc_fwd, dim3(nblk(int64_t(B) * out)), dim3(kBlk), 0, c->stream, c->h1,
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

int lsm_cnn_backward(lsm_cnn *c, const float *dy) {
    if (!c) return LSM_EINVAL;
    if (!c->bound || c->b_last < 1) return cfail(c, LSM_ESTATE, "forward first");
    const int B = int(c->b_last);
    const int hid = c->cfg.hidden, out = c->cfg.outputs, CL = c->C[kLayers];
    if (dy && dy != c->dy) CHIP(c, hipMemcpyAsync(c->dy, dy, size_t(B) * out * 4, hipMemcpyDeviceToDevice, c->stream));
    // dense layers
    hipLaunchKernelGGL(k_fc_bwd_weight, dim3(nblk(int64_t(out) * (hid + 1))), dim3(kBlk), 0, c->stream, c->dy, c->h1,
                       c->g + c->w_off[kLayers + 1], c->g + c->b_off[kLayers + 1], B, hid, out);
    hipLaunchKernelGGL(k_fc_bwd_data, dim3(nblk(int64_t(B) * hid)), dim3(kBlk), 0, c->stream, c->dy,
                       c->p + c->w_off[kLayers + 1], c->h1, c->dh1, B, hid, out);
    hipLaunchKernelGGL(k_fc_bwd_weight, dim3(nblk(int64_t(hid) * (CL + 1))), dim3(kBlk), 0, c->stream, c->dh1, c->gap,
                       c->g + c->w_off[kLayers], c->g + c->b_off[kLayers], B, CL, hid);
    hipLaunchKernelGGL(k_fc_bwd_data, dim3(nblk(int64_t(B) * CL)), dim3(kBlk), 0, c->stream, c->dh1,
                       c->p + c->w_off[kLayers], nullptr, c->dgap, B, CL, hid);
    CHIP(c, hipGetLastError());
    const int HL = c->Hs[kLayers - 1];
    hipLaunchKernelGGL(k_gap_bwd_relu, dim3(nblk(int64_t(B) * HL * HL * CL)), dim3(kBlk), 0, c->stream, c->dgap,
                       c->act[kLayers - 1], c->dact[kLayers - 1], B, HL * HL, CL);
    CHIP(c, hipGetLastError());
    for (int l = kLayers - 1; l >= 0; --l) {
        const int H = c->Hs[l];
        const int64_t npix = int64_t(B) * H * H;
        const int64_t sp = splits_for(npix);
        const int64_t nw = c->w_n[l], cout = c->C[l + 1], cin = c->C[l];
        if (l > 0) {
            // weight gradient: MFMA over pixel splits, then a fixed-order sum
            const dim3 grid(unsigned((cout + 63) / 64), unsigned(9 * ((cin + 63) / 64)), unsigned(sp));
            hipLaunchKernelGGL(k_conv_wgrad_mfma, grid, dim3(kBlk), 0, c->stream, c->pool[l - 1], c->dact[l], c->part,
                               B, H, H, int(cin), int(cout), int64_t(kSplitPix));
            CHIP(c, hipGetLastError());
            hipLaunchKernelGGL(k_sum_splits, dim3(nblk(nw)), dim3(kBlk), 0, c->stream, c->part, c->g + c->w_off[l], nw,
                               int(sp));
            // bias gradient
            hipLaunchKernelGGL(k_colsum_bf16, dim3(unsigned(sp)), dim3(kBlk), 0, c->stream, c->dact[l], c->part, npix,
                               int(cout), int64_t(kSplitPix));
            hipLaunchKernelGGL(k_sum_splits, dim3(nblk(cout)), dim3(kBlk), 0, c->stream, c->part, c->g + c->b_off[l],
                               cout, int(sp));
            CHIP(c, hipGetLastError());
            // input gradient: implicit GEMM with the flipped weights, then the
            // pooling and ReLU of the layer below
            const int64_t npin = npix;
            const dim3 g2(unsigned((npin + 64 * kConvWM - 1) / (64 * kConvWM)),
                          unsigned((cin + 16 * kConvWN - 1) / (16 * kConvWN)));
            hipLaunchKernelGGL((k_conv_mfma<false, kConvWM, kConvWN>), g2, dim3(kBlk), 0, c->stream, c->dact[l], c->wd[l], nullptr,
                               c->dpool[l - 1], B, H, H, int(cout), int(cin));
            CHIP(c, hipGetLastError());
            const int Hp = c->Hs[l - 1];
            hipLaunchKernelGGL(k_pool2_bwd_relu, dim3(nblk(int64_t(B) * Hp * Hp * cin)), dim3(kBlk), 0, c->stream,
                               c->dpool[l - 1], c->act[l - 1], c->dact[l - 1], B, Hp, Hp, int(cin));
            CHIP(c, hipGetLastError());
        } else {
            const unsigned groups = unsigned((cout / 8 + kBlk / 64 - 1) / (kBlk / 64));
            hipLaunchKernelGGL(k_conv1_wgrad, dim3(unsigned(sp), groups), dim3(kBlk), 0, c->stream, c->x_last,
                               c->dact[0], c->part, B, H, H, int(cout), int64_t(kSplitPix));
            // part layout [split][co][10]: taps then bias
            hipLaunchKernelGGL(k_sum_splits, dim3(nblk(cout * 10)), dim3(kBlk), 0, c->stream, c->part,
                               c->part + sp * cout * 10, cout * 10, int(sp));
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

int lsm_cnn_conv_forward(lsm_cnn *c, int layer, const void *in, void *out, int64_t batch) {
    // single layer of the implicit-GEMM convolution (layers 1..4) on caller
    // buffers, with this network's weights: used to test the kernel alone
    if (!c || !in || !out || layer < 1 || layer >= kLayers || batch < 1) return LSM_EINVAL;
    if (!c->bound) return cfail(c, LSM_ESTATE, "bind first");
    const int H = c->Hs[layer];
    const int64_t npix = batch * H * H;
    const dim3 grid(unsigned((npix + 64 * kConvWM - 1) / (64 * kConvWM)),
                    unsigned((c->C[layer + 1] + 16 * kConvWN - 1) / (16 * kConvWN)));
    hipLaunchKernelGGL((k_conv_mfma<true, kConvWM, kConvWN>), grid, dim3(kBlk), 0, c->stream, static_cast<const u16 *>(in), c->wf[layer],
                       c->p + c->b_off[layer], static_cast<u16 *>(out), int(batch), H, H, c->C[layer], c->C[layer + 1]);
    CHIP(c, hipGetLastError());
    return LSM_OK;
}

}  // extern "C"
