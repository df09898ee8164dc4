// Internal interface of the corrector kernels (lf_corrector.hip) used by the
// C-ABI runtime (lf_corrector_api.cpp). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lf {

constexpr int kCorrTileW = 16, kCorrTileH = 8;  // output pixels per conv workgroup
constexpr float kCorrWScale = 4.0f;             // input channel 3 = W / 4
constexpr float kCorrNScale = 8.0f;             // input channel 4 = n / 8
constexpr int kCorrParams = 20835;              // 1472 + 9248 + 9248 + 867

// One layer: real and padded channel counts, offsets of its packed weights.
struct CorrLayer {
    int32_t cin, cout;        // real channels
    int32_t cinp, coutp, kf;  // forward conv: padded input / output channels, reduction length
    int32_t cinp_b, coutp_b, kb;  // backward-data conv: outputs (= cin padded), inputs (= cout padded), reduction
    int32_t poff;             // offset of w (then b) in the flat FP32 parameters
    int32_t wf_off, wb_off;   // offsets (bf16 elements) of the forward / backward packed weights
    int32_t b_off;            // offset of the padded FP32 bias
};
struct CorrLayout {
    CorrLayer layer[4];
};

hipError_t corr_input(const float *rgb, const float *wsum, const uint8_t *count, int64_t P, uint16_t *a0,
                      hipStream_t s);
hipError_t corr_pack(const float *prm, const CorrLayout &L, uint16_t *wbuf, float *bbuf, hipStream_t s);
hipError_t corr_conv(int layer, bool backward, const uint16_t *in, int32_t N, int32_t H, int32_t W,
                     const uint16_t *wpk, const float *bias, void *out, const uint16_t *mask, hipStream_t s);
hipError_t corr_dw(int layer, const uint16_t *x, const uint16_t *dz, int32_t N, int32_t H, int32_t W,
                   int32_t cin_real, int32_t cout_real, float *partial, int slots, hipStream_t s);
hipError_t corr_reduce(const float *partial, int32_t slots, int32_t len, float *out, hipStream_t s);
hipError_t corr_loss(const float *rgb, const float *resid, const float *ref, int64_t P, uint16_t *dz,
                     float *loss_part, int blocks, hipStream_t s);
hipError_t corr_adam(float *prm, const float *grad, float *m1, float *m2, int32_t n, float lr, float b1, float b2,
                     float eps, float c1, float c2, hipStream_t s);
// Inference in one persistent kernel (all layers and the finish; grid workgroups).
hipError_t corr_fused(const float *rgb, const float *wsum, const uint8_t *count, int32_t N, int32_t H, int32_t W,
                      const uint16_t *wbuf, const float *bbuf, const CorrLayout &L, float thresh, float *out,
                      uint8_t *fb, float *resid_out, int grid, hipStream_t s);
int corr_fused_tiles(int32_t N, int32_t H, int32_t W);
hipError_t corr_fused_occupancy(int *per_cu);

}  // namespace lf
