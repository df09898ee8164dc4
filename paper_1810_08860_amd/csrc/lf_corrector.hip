// Learned residual corrector of the rendered eye view: four 3x3 convolutions
// (5 -> 32 -> 32 -> 32 -> 3 channels, ReLU after the first three, zero
// padding), output = render + residual, except pixels whose largest residual
// component exceeds a threshold keep the plain render. BF16 weights and
// activations, FP32 accumulation on MFMA (v_mfma_f32_16x16x32_bf16); FP32
// master weights trained with Adam by the kernels below.
//
// Convolution as an implicit GEMM: rows = output pixels (one 16-pixel run of
// an image row per MFMA block), columns = output channels, reduction =
// (tap, input channel) with the input channels of one tap contiguous. A
// workgroup computes a 16 x 8 pixel tile for every output channel from an
// LDS halo tile of the input and an LDS copy of the packed weights.
//
// Activation layout: NHWC, channels padded to a multiple of 8 (layer-1 input
// 8 = R, G, B, W/4, n/8, 0, 0, 0; hidden 32; residual FP32 x 4).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lf_corrector.h"

namespace lf {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Two FP32 values as packed BF16, a in the low half (hardware conversion,
// round to nearest even).
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b16x2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, b16x2));
}
__device__ __forceinline__ uint16_t f2bf(float f) { return (uint16_t)pack_bf16x2(f, 0.0f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int TW = kCorrTileW, TH = kCorrTileH;  // output tile: 16 x 8 pixels

template <int CIN>
constexpr int kpad() { return ((9 * CIN + 31) / 32) * 32; }

// ---------------------------------------------------------------------------------------------
// forward / backward-data convolution

enum { EPI_RELU_BF16 = 0, EPI_F32 = 1, EPI_MASK_BF16 = 2 };

// out = epilogue(conv3x3(in, w) [+ bias]) for one 16 x 8 tile per workgroup
// (256 threads: wave w owns tile rows 2w, 2w+1). CIN, COUT: padded channel
// counts of input and output (multiples of 8; COUT a multiple of 16 for the
// MFMA columns, COUT_ST the stored channel count).
template <int CIN, int COUT, int COUT_ST, int EPI>
__global__ __launch_bounds__(256) void k_conv(const uint16_t *__restrict__ in, int32_t N, int32_t H, int32_t W,
                                              const uint16_t *__restrict__ wpk, const float *__restrict__ bias,
                                              void *__restrict__ out, const uint16_t *__restrict__ mask) {
    constexpr int KP = kpad<CIN>();
    constexpr int NB = COUT / 16;
    constexpr int HX = TW + 2, HY = TH + 2;
    // pixel stride padded by 8 bf16 so that the 16 lanes of an A read hit
    // different LDS banks
    constexpr int PS = CIN + 8;
    __shared__ __attribute__((aligned(16))) uint16_t tin[HY * HX * PS];
    __shared__ __attribute__((aligned(16))) uint16_t tw[COUT * (KP + 8)];
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int b = blockIdx.x;
    const int n = b / (tiles_x * tiles_y), r = b % (tiles_x * tiles_y);
    const int x0 = (r % tiles_x) * TW, y0 = (r / tiles_x) * TH;
    const int tid = threadIdx.x;

    // weights: COUT rows of KP bf16, 16 bytes per thread and step
    for (int q = tid; q < COUT * KP / 8; q += 256) {
        const int row = q / (KP / 8), c8 = q % (KP / 8);
        *reinterpret_cast<uint4 *>(&tw[row * (KP + 8) + 8 * c8]) =
            *reinterpret_cast<const uint4 *>(&wpk[(int64_t)row * KP + 8 * c8]);
    }
    // input halo tile, zero outside the image
    for (int q = tid; q < HY * HX * (CIN / 8); q += 256) {
        const int pix = q / (CIN / 8), c8 = q % (CIN / 8);
        const int yy = y0 - 1 + pix / HX, xx = x0 - 1 + pix % HX;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (yy >= 0 && yy < H && xx >= 0 && xx < W)
            v = *reinterpret_cast<const uint4 *>(&in[(((int64_t)n * H + yy) * W + xx) * CIN + 8 * c8]);
        *reinterpret_cast<uint4 *>(&tin[pix * PS + 8 * c8]) = v;
    }
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63, i = lane & 15, g = lane >> 4;
    floatx4 acc[2][NB];
#pragma unroll
    for (int rr = 0; rr < 2; ++rr)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[rr][nb] = floatx4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int s = 0; s < KP / 32; ++s) {
        const int k0 = 32 * s + 8 * g;  // this lane's 8 reduction indices k0 .. k0+7
        const int t = k0 / CIN, ci = k0 % CIN;
        bf16x8 bv[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bv[nb] = *reinterpret_cast<const bf16x8 *>(&tw[(16 * nb + i) * (KP + 8) + k0]);
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            bf16x8 av = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
            if (t < 9) {
                const int ky = t / 3, kx = t % 3;
                const int row = 2 * wave + rr;
                av = *reinterpret_cast<const bf16x8 *>(&tin[((row + ky) * HX + i + kx) * PS + ci]);
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[rr][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bv[nb], av, acc[rr][nb], 0, 0, 0);
        }
    }

    // D[m][j] with the weights as the A operand: m = 4 g + v (output channel
    // in the block), j = i (pixel along the row), so each lane holds four
    // consecutive channels of one pixel and stores them at once
    const int xx = x0 + i;
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const int yy = y0 + 2 * wave + rr;
        if (yy >= H || xx >= W) continue;
        const int64_t p = ((int64_t)n * H + yy) * W + xx;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int c = 16 * nb + 4 * g;  // channels c .. c + 3
            if (c >= COUT_ST) continue;
            const floatx4 a = acc[rr][nb];
            if (EPI == EPI_RELU_BF16) {
                const float4 bi = *reinterpret_cast<const float4 *>(&bias[c]);
                *reinterpret_cast<uint2 *>(&reinterpret_cast<uint16_t *>(out)[p * COUT_ST + c]) =
                    make_uint2(pack_bf16x2(fmaxf(a[0] + bi.x, 0.0f), fmaxf(a[1] + bi.y, 0.0f)),
                               pack_bf16x2(fmaxf(a[2] + bi.z, 0.0f), fmaxf(a[3] + bi.w, 0.0f)));
            } else if (EPI == EPI_F32) {
                const float4 bi = *reinterpret_cast<const float4 *>(&bias[c]);
                *reinterpret_cast<float4 *>(&reinterpret_cast<float *>(out)[p * COUT_ST + c]) =
                    make_float4(a[0] + bi.x, a[1] + bi.y, a[2] + bi.z, a[3] + bi.w);
            } else {
                const uint2 mk = *reinterpret_cast<const uint2 *>(&mask[p * COUT_ST + c]);
                const float m0 = bf2f((uint16_t)mk.x), m1 = bf2f((uint16_t)(mk.x >> 16));
                const float m2 = bf2f((uint16_t)mk.y), m3 = bf2f((uint16_t)(mk.y >> 16));
                *reinterpret_cast<uint2 *>(&reinterpret_cast<uint16_t *>(out)[p * COUT_ST + c]) =
                    make_uint2(pack_bf16x2(m0 > 0.0f ? a[0] : 0.0f, m1 > 0.0f ? a[1] : 0.0f),
                               pack_bf16x2(m2 > 0.0f ? a[2] : 0.0f, m3 > 0.0f ? a[3] : 0.0f));
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// weight gradient: dW[t][ci][co] = sum_p x[p + d_t][ci] dz[p][co], db[co] = sum_p dz[p][co]
//
// GEMM with rows (t, ci), columns co and the reduction over pixels. A
// workgroup strides over 16 x 8 tiles, staging x (with halo, one copy per
// horizontal tap offset so that 8 consecutive pixels are one aligned 16-byte
// LDS read) and dz channel-major from 16-byte loads of 8 channels, and keeps
// its partial sums in registers; db is summed by all threads (channel t mod
// 32, every 8th pixel). At the end it writes its partial dW / db to its own
// slot (reduced in a fixed order by k_reduce_partials: deterministic).
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_dw(const uint16_t *__restrict__ x, const uint16_t *__restrict__ dz,
                                                 int32_t N, int32_t H, int32_t W, int32_t cin_real,
                                                 int32_t cout_real, float *__restrict__ partial) {
    static_assert(CIN % 8 == 0 && COUT % 8 == 0 && COUT <= 32, "channels come in 16-byte chunks");
    constexpr int MB = (9 * CIN + 15) / 16;  // row blocks of 16 (t, ci) pairs
    constexpr int NBK = (COUT + 15) / 16;
    constexpr int NBLK = MB * NBK;
    constexpr int PER = (NBLK + 3) / 4;      // output blocks per wave
    constexpr int HY = TH + 2, HX = TW + 2;  // x tile with its halo
    constexpr int CX = CIN / 8, CZ = COUT / 8;
    // channel planes padded by 16 bytes: the 16 lanes of an MFMA operand read
    // (consecutive channels) then start on different LDS banks
    constexpr int PX = HY * TW + 8, PZ = TH * TW + 8;
    __shared__ __attribute__((aligned(16))) uint16_t xs[3][CIN][PX];
    __shared__ __attribute__((aligned(16))) uint16_t dzs[16 * NBK][PZ];
    __shared__ float s_db[8][32];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, i = lane & 15, g = lane >> 4;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int total = N * tiles_x * tiles_y;
    floatx4 acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    float db_acc = 0.0f;  // channel tid % 32, pixels tid / 32 + 8 k of each tile
    // padding channels of dz (16 NBK > COUT) stay zero
    for (int q = tid; q < (16 * NBK - COUT) * PZ; q += 256) (&dzs[COUT][0])[q] = 0;

    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int n = tile / (tiles_x * tiles_y), r = tile % (tiles_x * tiles_y);
        const int x0 = (r % tiles_x) * TW, y0 = (r / tiles_x) * TH;
        __syncthreads();
        // x tile: xs[kx][c][row][col] = x[y0 - 1 + row][x0 + col + kx - 1][c]; a loaded
        // pixel at halo column hc lands in column hc - kx of copy kx
        for (int q = tid; q < HY * CX * HX; q += 256) {
            // a wave's lanes cover consecutive columns and rows of one chunk h
            const int hc = q % HX, row = (q / HX) % HY, h = q / (HX * HY);
            const int yy = y0 - 1 + row, xx = x0 - 1 + hc;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                v = *reinterpret_cast<const uint4 *>(&x[(((int64_t)n * H + yy) * W + xx) * CIN + 8 * h]);
            const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int col = hc - kx;
                if (col >= 0 && col < TW) {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        xs[kx][8 * h + e][row * TW + col] = (uint16_t)(wv[e >> 1] >> (16 * (e & 1)));
                }
            }
        }
        for (int q = tid; q < TH * CZ * TW; q += 256) {
            const int col = q % TW, row = (q / TW) % TH, h = q / (TW * TH);
            const int yy = y0 + row, xx = x0 + col;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (yy < H && xx < W) v = *reinterpret_cast<const uint4 *>(&dz[(((int64_t)n * H + yy) * W + xx) * COUT + 8 * h]);
            const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) dzs[8 * h + e][row * TW + col] = (uint16_t)(wv[e >> 1] >> (16 * (e & 1)));
        }
        __syncthreads();
        if ((tid & 31) < COUT) {
            const int c = tid & 31;
            float sacc = 0.0f;
#pragma unroll
            for (int k = 0; k < TH * TW / 8; ++k) {
                const int p = (tid >> 5) + 8 * k;
                sacc += bf2f(dzs[c][p]);
            }
            db_acc += sacc;
        }
        // reduction over the tile's 128 pixels in 4 steps of 32 (two rows of 16)
#pragma unroll
        for (int s = 0; s < TH / 2; ++s) {
            const int row = 2 * s + (g >> 1), col = 8 * (g & 1);
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int blk = wave * PER + q;
                if (blk >= NBLK) continue;
                const int mb = blk / NBK, nb = blk % NBK;
                const int m = 16 * mb + i;  // (t, ci) row of this lane
                bf16x8 av = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
                if (m < 9 * CIN) {
                    const int t = m / CIN, ci = m % CIN;
                    const int ky = t / 3, kx = t % 3;
                    av = *reinterpret_cast<const bf16x8 *>(&xs[kx][ci][(row + ky) * TW + col]);
                }
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&dzs[16 * nb + i][row * TW + col]);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[q], 0, 0, 0);
            }
        }
    }
    // partial result of this workgroup in the flat parameter layout (dw then db)
    const int nw = 9 * cin_real * cout_real;
    float *pw = partial + (int64_t)blockIdx.x * (nw + cout_real);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int blk = wave * PER + q;
        if (blk >= NBLK) continue;
        const int mb = blk / NBK, nb = blk % NBK;
        const int co = 16 * nb + i;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = 16 * mb + 4 * g + v;
            if (m >= 9 * CIN) continue;
            const int t = m / CIN, ci = m % CIN;
            if (ci < cin_real && co < cout_real) pw[(t * cin_real + ci) * cout_real + co] = acc[q][v];
        }
    }
    s_db[tid >> 5][tid & 31] = db_acc;
    __syncthreads();
    if (tid < cout_real) {
        float d = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) d += s_db[k][tid];
        pw[nw + tid] = d;
    }
}

// out[j] = sum over slots of partial[slot][j], in a fixed order: a workgroup
// covers 64 consecutive j; its 4 waves each sum every 4th slot with 8
// independent accumulators (8 loads in flight per lane), and the 4 x 8 partial
// sums of each j are then added in one fixed order.
__global__ __launch_bounds__(256) void k_reduce_partials(const float *__restrict__ partial, int32_t slots,
                                                         int32_t len, float *__restrict__ out) {
    __shared__ float part[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (j < len) {
        int k = wave;
        for (; k + 28 < slots; k += 32) {
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += partial[(int64_t)(k + 4 * u) * len + j];
        }
        for (int u = 0; k < slots; k += 4, ++u) acc[u & 7] += partial[(int64_t)k * len + j];
    }
    part[wave][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    if (wave == 0 && j < len) out[j] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// ---------------------------------------------------------------------------------------------
// element-wise pieces

// Layer-1 input: (R, G, B, W / 4, n / 8, 0, 0, 0) in BF16.
__global__ void k_corr_input(const float *__restrict__ rgb, const float *__restrict__ wsum,
                             const uint8_t *__restrict__ count, int64_t P, uint16_t *__restrict__ a0) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        uint16_t v[8];
        v[0] = f2bf(rgb[3 * p]);
        v[1] = f2bf(rgb[3 * p + 1]);
        v[2] = f2bf(rgb[3 * p + 2]);
        v[3] = f2bf(wsum[p] * (1.0f / kCorrWScale));
        v[4] = f2bf((float)count[p] * (1.0f / kCorrNScale));
        v[5] = v[6] = v[7] = 0;
        uint4 o;
        o.x = v[0] | ((uint32_t)v[1] << 16);
        o.y = v[2] | ((uint32_t)v[3] << 16);
        o.z = v[4];
        o.w = 0;
        reinterpret_cast<uint4 *>(a0)[p] = o;
    }
}

// Training loss: diff = render + residual - ref; partial sums of diff^2 per
// block, and dL/d(residual) = 2 diff / (3P) in BF16 (8-channel layout).
__global__ __launch_bounds__(256) void k_corr_loss(const float *__restrict__ rgb, const float *__restrict__ resid,
                                                   const float *__restrict__ ref, int64_t P,
                                                   uint16_t *__restrict__ dz, float *__restrict__ loss_part) {
    __shared__ float red[256];
    float s = 0.0f;
    const float k = 2.0f / (3.0f * (float)P);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        uint16_t d[3];
        for (int c = 0; c < 3; ++c) {
            const float df = rgb[3 * p + c] + resid[4 * p + c] - ref[3 * p + c];
            s += df * df;
            d[c] = f2bf(k * df);
        }
        uint4 o;
        o.x = d[0] | ((uint32_t)d[1] << 16);
        o.y = d[2];
        o.z = 0;
        o.w = 0;
        reinterpret_cast<uint4 *>(dz)[p] = o;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Adam on the FP32 master parameters.
__global__ void k_adam(float *__restrict__ prm, const float *__restrict__ grad, float *__restrict__ m1,
                       float *__restrict__ m2, int32_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = grad[j];
    const float a = b1 * m1[j] + (1.0f - b1) * gj;
    const float v = b2 * m2[j] + (1.0f - b2) * gj * gj;
    m1[j] = a;
    m2[j] = v;
    prm[j] -= lr * (a * c1) / (sqrtf(v * c2) + eps);
}

// Pack the FP32 master parameters of every layer into the MFMA layouts:
// forward wf[co][t * CINP + ci] (zero padded), FP32 bias, and for the
// backward-data pass wb[ci][t' * COUTP_in + co] = w[8 - t'][ci][co].
__global__ void k_corr_pack(const float *__restrict__ prm, CorrLayout L, uint16_t *__restrict__ wbuf,
                            float *__restrict__ bbuf) {
    const int layer = blockIdx.y;
    const CorrLayer &ly = L.layer[layer];
    const float *w = prm + ly.poff;
    const float *b = w + 9 * ly.cin * ly.cout;
    const int nf = ly.coutp * ly.kf, nb = ly.cinp_b * ly.kb;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nf + nb + ly.coutp; q += gridDim.x * blockDim.x) {
        if (q < nf) {
            const int co = q / ly.kf, k = q % ly.kf, t = k / ly.cinp, ci = k % ly.cinp;
            float v = 0.0f;
            if (t < 9 && ci < ly.cin && co < ly.cout) v = w[(t * ly.cin + ci) * ly.cout + co];
            wbuf[ly.wf_off + q] = f2bf(v);
        } else if (q < nf + nb) {
            const int qq = q - nf;
            const int ci = qq / ly.kb, k = qq % ly.kb, tp = k / ly.coutp_b, co = k % ly.coutp_b;
            float v = 0.0f;
            if (tp < 9 && ci < ly.cin && co < ly.cout) v = w[((8 - tp) * ly.cin + ci) * ly.cout + co];
            wbuf[ly.wb_off + qq] = f2bf(v);
        } else {
            const int co = q - nf - nb;
            bbuf[ly.b_off + co] = co < ly.cout ? b[co] : 0.0f;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// fused inference: all four layers and the finish in one kernel
//
// A persistent workgroup takes 16 x 16 output tiles. The layer-1 input is
// built straight from the render (R, G, B, W / 4, n / 8, zero outside the
// image) over the tile grown by 4 pixels per side; each layer then computes
// its output over a region one pixel smaller per side (22^2, 20^2, 18^2,
// 16^2), entirely in LDS, with activations outside the image set to zero as
// the per-layer zero padding requires. The weights are the MFMA's A operand:
// every lane holds its fragments of layers 2 and 3 in registers for the life
// of the workgroup, and fetches those of layers 1 and 4 (cached) at the start
// of each use, so LDS traffic is the activations only. Regions are linearised
// row-major and cut into 16-pixel MFMA row blocks, which a wave takes two at a
// time; K-steps and packing match k_conv, so each layer accumulates in the
// same order as the layer-by-layer path. The tile's own FP32 render values
// stay in LDS (in the layer-1 input's space once layer 1 has read it) for the
// final blend, so the next tile's inputs can be fetched into registers during
// layers 2-4. Each XCD takes a contiguous range of tiles (shared halos stay in
// its L2).
constexpr int FT = 16;                                   // output tile side
constexpr int FR0 = FT + 8, FR1 = FT + 6, FR2 = FT + 4, FR3 = FT + 2;
constexpr int FPS = 40;                                  // hidden pixel stride: 32 channels + 8 pad

// ReLU of two packed BF16 values: a BF16 value is negative exactly when its
// bits read as a negative 16-bit integer, so one packed integer maximum with
// zero does it (and rounding to BF16 keeps the sign, so this equals rounding
// the ReLU of the FP32 values; a NaN with its sign bit set becomes 0 and
// one without stays NaN, where fmaxf gives 0 for both).
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t p) {
    typedef short s16x2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p), (s16x2){0, 0}));
}

// Activation tiles are addressed through LDS (address space 3) pointers, so
// index arithmetic stays 32-bit.
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) bf16x8 lds_bf16x8;

// a * b for a, b below 2^24 as one 24-bit multiply. Written out because the
// compiler otherwise folds a 32-bit multiply and the following add into a
// 64-bit multiply-add whose unused high addend register can alias the
// destination of an outstanding global load, which makes the wave wait for
// every load in flight (the next tile's prefetch).
__device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "s"(b), "v"(a));
    return r;
}

template <int SOUT, bool IN8>
__device__ __forceinline__ uint32_t fused_base(int x, int y, int g) {
    constexpr int SIN = SOUT + 2;
    // element index of this lane's first K-step operand; 24-bit products
    return IN8 ? mul24((uint32_t)(y * SIN + x), 8u) : mul24((uint32_t)(y * SIN + x), (uint32_t)FPS) + 8u * g;
}

template <int SOUT, bool IN8>
__device__ __forceinline__ bf16x8 fused_a(const lds_u16 *__restrict__ src, uint32_t base, int s, int g) {
    constexpr int SIN = SOUT + 2;
    bf16x8 av = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (IN8) {
        // four taps of 8 channels per K-step; the padding taps 9-11 carry zero
        // weights, so they read tap 8's (finite) activations instead of a branch
        const int t = min(4 * s + g, 8);
        av = *reinterpret_cast<const lds_bf16x8 *>(&src[base + ((t / 3) * SIN + t % 3) * 8]);
    } else {
        av = *reinterpret_cast<const lds_bf16x8 *>(&src[base + ((s / 3) * SIN + s % 3) * FPS]);
    }
    return av;
}

// The accumulators already hold the bias (fused_bias). interior: the tile's
// whole region lies inside the image, so no activation needs the zero of the
// per-layer padding.
template <int SOUT, int NBO, bool LAST>
__device__ __forceinline__ void fused_store(const floatx4 (&acc)[NBO], int mm, uint16_t *__restrict__ dst,
                                            float *__restrict__ res, bool interior, int ox0, int oy0, int H, int W,
                                            int g) {
    constexpr int NOUT = SOUT * SOUT;
    if (mm >= NOUT) return;
    const int x = mm % SOUT, y = mm / SOUT;
    const int xx = ox0 + x, yy = oy0 + y;
    const bool in = interior || (xx >= 0 && xx < W && yy >= 0 && yy < H);
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) f32x4 lds_f32x4;
    typedef __attribute__((address_space(3))) u32x2 lds_u32x2;
    const uint32_t o0 = mul24((uint32_t)mm, (uint32_t)FPS) + 4u * g;
#pragma unroll
    for (int nb = 0; nb < NBO; ++nb) {
        const float v0 = acc[nb][0], v1 = acc[nb][1], v2 = acc[nb][2], v3 = acc[nb][3];
        if (LAST) {
            if (g == 0)
                *reinterpret_cast<lds_f32x4 *>(&((__attribute__((address_space(3))) float *)res)[4u * mm]) =
                    f32x4{v0, v1, v2, v3};
        } else {
            u32x2 o = u32x2{0u, 0u};
            if (in) o = u32x2{relu_bf16x2(pack_bf16x2(v0, v1)), relu_bf16x2(pack_bf16x2(v2, v3))};
            *reinterpret_cast<lds_u32x2 *>(&((lds_u16 *)dst)[o0 + 16 * nb]) = o;
        }
    }
}

// Accumulator start values: the bias of this lane's four output channels
// (channel 16 nb + 4 g + v sits in element v of block nb's D fragment).
template <int NBO>
__device__ __forceinline__ void fused_bias(floatx4 (&acc)[NBO], const float *__restrict__ s_bias, int g) {
#pragma unroll
    for (int nb = 0; nb < NBO; ++nb) {
        const float4 bi = *reinterpret_cast<const float4 *>(&s_bias[16 * nb + 4 * g]);
        acc[nb] = floatx4{bi.x, bi.y, bi.z, bi.w};
    }
}

// One hidden layer (or the last): output region side SOUT from the input
// region side SOUT + 2; IN8: 8-channel layer-1 input; NBO blocks of 16 output
// channels. The weights are the MFMA's A operand and the activations its B
// operand, so D[4 g + v][i] is channel 16 nb + 4 g + v of pixel 16 b + i:
// each lane stores four consecutive channels of one pixel at once.
// PAIR: a wave takes two 16-pixel blocks at a time (blocks b and b + 4), four
// independent accumulation chains. Each K-step's activations are read from
// LDS one step ahead of the MFMAs that use them, and scheduling barriers keep
// the compiler from hoisting further reads (registers: two layers' weights
// live in them for the whole kernel).
template <int SOUT, bool IN8, int KS, int NBO, bool LAST, bool PAIR>
__device__ __forceinline__ void fused_layer(const uint16_t *__restrict__ src, uint16_t *__restrict__ dst,
                                            float *__restrict__ res, const bf16x8 (&w)[KS][NBO],
                                            const float *__restrict__ s_bias, bool interior, int ox0, int oy0, int H,
                                            int W) {
    constexpr int NOUT = SOUT * SOUT, NBLK = (NOUT + 15) / 16;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, i = lane & 15, g = lane >> 4;
    const lds_u16 *s3 = (const lds_u16 *)src;
    for (int b = wave; b < NBLK; b += PAIR ? 8 : 4) {
        const int mm0 = 16 * b + i, mm1 = mm0 + 64;  // this lane's pixels (block b, block b + 4)
        const int m0 = min(mm0, NOUT - 1);
        const uint32_t q0 = fused_base<SOUT, IN8>(m0 % SOUT, m0 / SOUT, g);
        if (PAIR && b + 4 < NBLK) {
            const int m1 = min(mm1, NOUT - 1);
            const uint32_t q1 = fused_base<SOUT, IN8>(m1 % SOUT, m1 / SOUT, g);
            floatx4 acc0[NBO], acc1[NBO];
            fused_bias<NBO>(acc0, s_bias, g);
            fused_bias<NBO>(acc1, s_bias, g);
            bf16x8 a0 = fused_a<SOUT, IN8>(s3, q0, 0, g), a1 = fused_a<SOUT, IN8>(s3, q1, 0, g);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const bf16x8 c0 = a0, c1 = a1;
                if (s + 1 < KS) {
                    a0 = fused_a<SOUT, IN8>(s3, q0, s + 1, g);
                    a1 = fused_a<SOUT, IN8>(s3, q1, s + 1, g);
                }
#pragma unroll
                for (int nb = 0; nb < NBO; ++nb) {
                    acc0[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[s][nb], c0, acc0[nb], 0, 0, 0);
                    acc1[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[s][nb], c1, acc1[nb], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            fused_store<SOUT, NBO, LAST>(acc0, mm0, dst, res, interior, ox0, oy0, H, W, g);
            fused_store<SOUT, NBO, LAST>(acc1, mm1, dst, res, interior, ox0, oy0, H, W, g);
        } else {
            floatx4 acc[NBO];
            fused_bias<NBO>(acc, s_bias, g);
            bf16x8 a0 = fused_a<SOUT, IN8>(s3, q0, 0, g);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const bf16x8 c0 = a0;
                if (s + 1 < KS) a0 = fused_a<SOUT, IN8>(s3, q0, s + 1, g);
#pragma unroll
                for (int nb = 0; nb < NBO; ++nb)
                    acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[s][nb], c0, acc[nb], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
            fused_store<SOUT, NBO, LAST>(acc, mm0, dst, res, interior, ox0, oy0, H, W, g);
        }
    }
}

// Two workgroups per CU (each 80 KB of LDS and at most 256 registers per
// lane) so that one's global loads and barriers overlap the other's MFMAs.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_corr_fused(const float *__restrict__ rgb, const float *__restrict__ wsum,
                                                    const uint8_t *__restrict__ count, int32_t N, int32_t H,
                                                    int32_t W, const uint16_t *__restrict__ wbuf,
                                                    const float *__restrict__ bbuf, CorrLayout L, float thresh,
                                                    float *__restrict__ out, uint8_t *__restrict__ fb,
                                                    float *__restrict__ resid_out) {
    __shared__ __attribute__((aligned(16))) uint16_t s_in[FR0 * FR0 * 8];
    __shared__ __attribute__((aligned(16))) uint16_t s_a[FR1 * FR1 * FPS];  // layer 1, then layer 3
    __shared__ __attribute__((aligned(16))) uint16_t s_b[FR2 * FR2 * FPS];  // layer 2, then the residual
    __shared__ __attribute__((aligned(16))) float s_bias[4][32];
    float *s_res = reinterpret_cast<float *>(s_b);
    // the tile's own render values (FP32 RGB of its 16 x 16 pixels), kept in
    // s_in's space once layer 1 has read it, for the final blend
    float *s_rgb = reinterpret_cast<float *>(s_in);
    static_assert(sizeof(s_in) >= FT * FT * 3 * sizeof(float), "stash fits in the layer-1 input");
    const int tid = threadIdx.x, lane = tid & 63, i = lane & 15, g = lane >> 4;

    // padded biases of the four layers
    if (tid < 128) {
        const int l = tid >> 5, c = tid & 31;
        s_bias[l][c] = (l < 3 || c < 16) ? bbuf[L.layer[l].b_off + c] : 0.0f;
    }
    // this lane's weight fragments of layers 2-3 (row 16 nb + i, columns
    // 32 s + 8 g ..), held for the life of the workgroup; layers 1 and 4's
    // are fetched per tile (cached), which leaves registers for the prefetch
    // below and for two blocks in flight per wave
    bf16x8 w2[9][2], w3[9][2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const int co = 16 * nb + i;
#pragma unroll
        for (int s = 0; s < 9; ++s) {
            w2[s][nb] = *reinterpret_cast<const bf16x8 *>(&wbuf[L.layer[1].wf_off + co * L.layer[1].kf + 32 * s + 8 * g]);
            w3[s][nb] = *reinterpret_cast<const bf16x8 *>(&wbuf[L.layer[2].wf_off + co * L.layer[2].kf + 32 * s + 8 * g]);
        }
    }

    const int tx = (W + FT - 1) / FT, ty = (H + FT - 1) / FT;
    const int total = N * tx * ty;
    // The layer-1 inputs of a tile (its region grown by 4 pixels per side) are
    // read from the render into registers one tile ahead: thread t holds
    // region pixels t, t + 256 and t + 512, and the next tile's loads are in
    // flight while this tile's layers run.
    constexpr int QN = (FR0 * FR0 + 255) / 256;
    float pr[QN], pg[QN], pb[QN], pw[QN];
    uint32_t pn[QN];
    auto fetch = [&](int t) {
        const int n = t / (tx * ty), r = t % (tx * ty);
        const int x0 = (r % tx) * FT, y0 = (r / tx) * FT;
        const int64_t img = (int64_t)n * H * W;
#pragma unroll
        for (int k = 0; k < QN; ++k) {
            const int q = tid + 256 * k;
            const int xx = x0 - 4 + q % FR0, yy = y0 - 4 + q / FR0;
            pr[k] = pg[k] = pb[k] = pw[k] = 0.0f;
            pn[k] = 0u;
            if (q < FR0 * FR0 && xx >= 0 && xx < W && yy >= 0 && yy < H) {
                const int64_t p = img + (int64_t)yy * W + xx;
                pr[k] = rgb[3 * p];
                pg[k] = rgb[3 * p + 1];
                pb[k] = rgb[3 * p + 2];
                pw[k] = wsum[p];
                pn[k] = count[p];
            }
        }
    };
    // Workgroup b runs on XCD b mod 8 (when the grid is a multiple of 8): each
    // XCD takes one contiguous eighth of the tiles, so neighbouring tiles, whose
    // inputs overlap by the 4-pixel halo, meet in the same L2.
    const bool by_xcd = gridDim.x % 8 == 0;
    const int stride = by_xcd ? gridDim.x / 8 : gridDim.x;
    const int t_lo = by_xcd ? (int)((int64_t)total * (blockIdx.x % 8) / 8) : 0;
    const int t_hi = by_xcd ? (int)((int64_t)total * (blockIdx.x % 8 + 1) / 8) : total;
    const int t_first = t_lo + (by_xcd ? blockIdx.x / 8 : blockIdx.x);
    if (t_first < t_hi) fetch(t_first);
    for (int tile = t_first; tile < t_hi; tile += stride) {
        const int n = tile / (tx * ty), r = tile % (tx * ty);
        const int x0 = (r % tx) * FT, y0 = (r / tx) * FT;
        const int64_t img = (int64_t)n * H * W;
        // layer-1 input (R, G, B, W / 4, n / 8; zero outside the image) from the staged values
#pragma unroll
        for (int k = 0; k < QN; ++k) {
            const int q = tid + 256 * k;
            if (q < FR0 * FR0) {
                uint4 o;
                o.x = pack_bf16x2(pr[k], pg[k]);
                o.y = pack_bf16x2(pb[k], pw[k] * (1.0f / kCorrWScale));
                o.z = pack_bf16x2((float)pn[k] * (1.0f / kCorrNScale), 0.0f);
                o.w = 0u;
                *reinterpret_cast<uint4 *>(&s_in[q * 8]) = o;
            }
        }
        // (an opaque zero offset keeps the compiler from hoisting these loads
        // out of the tile loop, which would keep them live across it)
        int wz = 0;
        asm volatile("" : "+s"(wz));
        bf16x8 w1[3][2];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int s = 0; s < 3; ++s)
                w1[s][nb] = *reinterpret_cast<const bf16x8 *>(
                    &wbuf[wz + L.layer[0].wf_off + (16 * nb + i) * L.layer[0].kf + 32 * s + 8 * g]);
        __syncthreads();
        // the layer-1 input region (4 pixels of margin) inside the image: no padding zeros anywhere
        const bool interior = x0 >= 4 && y0 >= 4 && x0 + FT + 4 <= W && y0 + FT + 4 <= H;
        fused_layer<FR1, true, 3, 2, false, true>(s_in, s_a, nullptr, w1, s_bias[0], interior, x0 - 3, y0 - 3, H, W);
        __syncthreads();
        // s_in is free: keep this tile's render values for the blend, then
        // fetch the next tile's inputs into the registers that held them
#pragma unroll
        for (int k = 0; k < QN; ++k) {
            const int q = tid + 256 * k;
            const int cx = q % FR0 - 4, cy = q / FR0 - 4;
            if (q < FR0 * FR0 && cx >= 0 && cx < FT && cy >= 0 && cy < FT) {
                float *d = &s_rgb[(cy * FT + cx) * 3];
                d[0] = pr[k];
                d[1] = pg[k];
                d[2] = pb[k];
            }
        }
        if (tile + stride < t_hi) fetch(tile + stride);
        fused_layer<FR2, false, 9, 2, false, true>(s_a, s_b, nullptr, w2, s_bias[1], interior, x0 - 2, y0 - 2, H, W);
        __syncthreads();
        fused_layer<FR3, false, 9, 2, false, true>(s_b, s_a, nullptr, w3, s_bias[2], interior, x0 - 1, y0 - 1, H, W);
        __syncthreads();
        {
            int wz4 = 0;
            asm volatile("" : "+s"(wz4));
            bf16x8 w4[9][1];
#pragma unroll
            for (int s = 0; s < 9; ++s)
                w4[s][0] = *reinterpret_cast<const bf16x8 *>(&wbuf[wz4 + L.layer[3].wf_off + i * L.layer[3].kf + 32 * s + 8 * g]);
            fused_layer<FT, false, 9, 1, true, true>(s_a, nullptr, s_res, w4, s_bias[3], interior, x0, y0, H, W);
        }
        // finish: out = render + residual, or the render where max |residual| > thresh.
        // Layer 4's block b is tile row b, computed by wave b mod 4: each wave
        // finishes its own rows (w, w + 4, w + 8, w + 12), so only its own LDS
        // writes need to be complete
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
        {
            const int px = (((tid >> 6) + 4 * ((tid & 63) >> 4)) << 4) + (tid & 15);
            const int xx = x0 + (px & 15), yy = y0 + (px >> 4);
            if (xx < W && yy < H) {
                const int64_t p = img + (int64_t)yy * W + xx;
                const float r0 = s_res[px * 4], r1 = s_res[px * 4 + 1], r2 = s_res[px * 4 + 2];
                const bool f = fmaxf(fabsf(r0), fmaxf(fabsf(r1), fabsf(r2))) > thresh;
                const float c0 = s_rgb[px * 3], c1 = s_rgb[px * 3 + 1], c2 = s_rgb[px * 3 + 2];
                out[3 * p] = f ? c0 : c0 + r0;
                out[3 * p + 1] = f ? c1 : c1 + r1;
                out[3 * p + 2] = f ? c2 : c2 + r2;
                if (fb) fb[p] = f ? 1 : 0;
                if (resid_out) {
                    resid_out[3 * p] = r0;
                    resid_out[3 * p + 1] = r1;
                    resid_out[3 * p + 2] = r2;
                }
            }
        }
        __syncthreads();  // s_res (aliasing s_b) is read before the next tile's layer 2 writes s_b
    }
}

// ---------------------------------------------------------------------------------------------
// launchers

static int grid_elems(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

hipError_t corr_input(const float *rgb, const float *wsum, const uint8_t *count, int64_t P, uint16_t *a0,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_corr_input, dim3(grid_elems(P)), dim3(256), 0, s, rgb, wsum, count, P, a0);
    return hipGetLastError();
}

hipError_t corr_pack(const float *prm, const CorrLayout &L, uint16_t *wbuf, float *bbuf, hipStream_t s) {
    hipLaunchKernelGGL(k_corr_pack, dim3(64, 4), dim3(256), 0, s, prm, L, wbuf, bbuf);
    return hipGetLastError();
}

// Forward layer l (0..3) or backward-data pass of layer l (1..3: dz_l -> dz_{l-1}).
hipError_t corr_conv(int layer, bool backward, const uint16_t *in, int32_t N, int32_t H, int32_t W,
                     const uint16_t *wpk, const float *bias, void *out, const uint16_t *mask, hipStream_t s) {
    const int tiles = N * ((W + TW - 1) / TW) * ((H + TH - 1) / TH);
    const dim3 g(tiles), b(256);
    if (!backward) {
        switch (layer) {
        case 0: hipLaunchKernelGGL((k_conv<8, 32, 32, EPI_RELU_BF16>), g, b, 0, s, in, N, H, W, wpk, bias, out, mask); break;
        case 1:
        case 2: hipLaunchKernelGGL((k_conv<32, 32, 32, EPI_RELU_BF16>), g, b, 0, s, in, N, H, W, wpk, bias, out, mask); break;
        default: hipLaunchKernelGGL((k_conv<32, 16, 4, EPI_F32>), g, b, 0, s, in, N, H, W, wpk, bias, out, mask); break;
        }
    } else {
        switch (layer) {
        case 3: hipLaunchKernelGGL((k_conv<8, 32, 32, EPI_MASK_BF16>), g, b, 0, s, in, N, H, W, wpk, bias, out, mask); break;
        default: hipLaunchKernelGGL((k_conv<32, 32, 32, EPI_MASK_BF16>), g, b, 0, s, in, N, H, W, wpk, bias, out, mask); break;
        }
    }
    return hipGetLastError();
}

hipError_t corr_dw(int layer, const uint16_t *x, const uint16_t *dz, int32_t N, int32_t H, int32_t W,
                   int32_t cin_real, int32_t cout_real, float *partial, int slots, hipStream_t s) {
    switch (layer) {
    case 0: hipLaunchKernelGGL((k_conv_dw<8, 32>), dim3(slots), dim3(256), 0, s, x, dz, N, H, W, cin_real, cout_real, partial); break;
    case 1:
    case 2: hipLaunchKernelGGL((k_conv_dw<32, 32>), dim3(slots), dim3(256), 0, s, x, dz, N, H, W, cin_real, cout_real, partial); break;
    default: hipLaunchKernelGGL((k_conv_dw<32, 8>), dim3(slots), dim3(256), 0, s, x, dz, N, H, W, cin_real, cout_real, partial); break;
    }
    return hipGetLastError();
}

hipError_t corr_reduce(const float *partial, int32_t slots, int32_t len, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3((len + 63) / 64), dim3(256), 0, s, partial, slots, len, out);
    return hipGetLastError();
}

hipError_t corr_loss(const float *rgb, const float *resid, const float *ref, int64_t P, uint16_t *dz,
                     float *loss_part, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_corr_loss, dim3(blocks), dim3(256), 0, s, rgb, resid, ref, P, dz, loss_part);
    return hipGetLastError();
}

hipError_t corr_adam(float *prm, const float *grad, float *m1, float *m2, int32_t n, float lr, float b1, float b2,
                     float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, prm, grad, m1, m2, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t corr_fused(const float *rgb, const float *wsum, const uint8_t *count, int32_t N, int32_t H, int32_t W,
                      const uint16_t *wbuf, const float *bbuf, const CorrLayout &L, float thresh, float *out,
                      uint8_t *fb, float *resid_out, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_corr_fused, dim3(grid), dim3(256), 0, s, rgb, wsum, count, N, H, W, wbuf, bbuf, L, thresh,
                       out, fb, resid_out);
    return hipGetLastError();
}

int corr_fused_tiles(int32_t N, int32_t H, int32_t W) { return N * ((W + FT - 1) / FT) * ((H + FT - 1) / FT); }

hipError_t corr_fused_occupancy(int *per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (const void *)k_corr_fused, 256, 0);
}

}  // namespace lf
