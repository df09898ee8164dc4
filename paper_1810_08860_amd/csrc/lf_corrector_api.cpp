// C ABI of the learned residual corrector (include/lf.h): parameters,
// inference with per-pixel fallback, and one training step (forward, MSE
// loss, backward on MFMA, Adam) on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/lf.h"
#include "lf_corrector.h"
#include "lf_internal.h"

using namespace lf;

namespace {

int cfail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return fail_msg(code, buf);
}

#define CF_HIP(call, what)                                                                              \
    do {                                                                                                \
        hipError_t _e = (call);                                                                         \
        if (_e != hipSuccess)                                                                           \
            return cfail(_e == hipErrorOutOfMemory ? LF_ENOMEM : LF_EHIP, "%s: %s", what, hipGetErrorString(_e)); \
    } while (0)

// A byte range of a caller buffer (null pointers never overlap anything).
struct Span {
    const void *p;
    int64_t bytes;
};
bool overlaps(const Span &a, const Span &b) {
    if (!a.p || !b.p) return false;
    const uintptr_t a0 = (uintptr_t)a.p, b0 = (uintptr_t)b.p;
    return a0 < b0 + (uintptr_t)b.bytes && b0 < a0 + (uintptr_t)a.bytes;
}

constexpr int kDwSlots = 512;   // workgroups (and partial-sum slots) of a weight-gradient pass
constexpr int kLossBlocks = 1024;

int kpad(int c) { return ((9 * c + 31) / 32) * 32; }

CorrLayout make_layout() {
    CorrLayout L;
    const int cin[4] = {5, 32, 32, 32}, cout[4] = {32, 32, 32, 3};
    const int cinp[4] = {8, 32, 32, 32}, coutp[4] = {32, 32, 32, 16};
    const int coutp_b[4] = {32, 32, 32, 8};
    int poff = 0, woff = 0, boff = 0;
    for (int l = 0; l < 4; ++l) {
        CorrLayer &y = L.layer[l];
        y.cin = cin[l];
        y.cout = cout[l];
        y.cinp = cinp[l];
        y.coutp = coutp[l];
        y.kf = kpad(cinp[l]);
        y.cinp_b = cinp[l];
        y.coutp_b = coutp_b[l];
        y.kb = kpad(coutp_b[l]);
        y.poff = poff;
        poff += 9 * cin[l] * cout[l] + cout[l];
        y.wf_off = woff;
        woff += y.coutp * y.kf;
        y.wb_off = woff;
        woff += y.cinp_b * y.kb;
        y.b_off = boff;
        boff += y.coutp;
    }
    return L;
}

}  // namespace

struct lf_corrector {
    CorrLayout L = make_layout();
    float *prm = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;  // FP32 [kCorrParams]
    uint16_t *wbuf = nullptr;  // packed BF16 weights (forward + backward-data) of all layers
    float *bbuf = nullptr;     // padded FP32 biases
    bool packed = false;
    int64_t step = 0;
    // activations and gradients, grown on demand (P pixels)
    int64_t cap_px = 0;
    uint16_t *a[4] = {nullptr, nullptr, nullptr, nullptr};  // a0 (8 ch), a1..a3 (32 ch)
    float *resid = nullptr;                                   // [P][4]
    uint16_t *dz3 = nullptr;                                  // [P][8]
    uint16_t *dzA = nullptr, *dzB = nullptr;                  // [P][32]
    float *partial = nullptr;
    float *loss_part = nullptr;
    int fused_grid = 0;  // resident workgroups of the fused inference kernel (CUs x per CU)
};

namespace {

size_t wbuf_elems(const CorrLayout &L) {
    const CorrLayer &y = L.layer[3];
    return (size_t)y.wb_off + (size_t)y.cinp_b * y.kb;
}

int ensure_px(lf_corrector *c, int64_t P) {
    if (P <= c->cap_px) return LF_OK;
    (void)hipDeviceSynchronize();
    for (auto &p : c->a) {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    for (void *p : {(void *)c->resid, (void *)c->dz3, (void *)c->dzA, (void *)c->dzB})
        if (p) (void)hipFree(p);
    c->resid = nullptr;
    c->dz3 = c->dzA = c->dzB = nullptr;
    c->cap_px = 0;
    CF_HIP(hipMalloc(&c->a[0], (size_t)P * 8 * 2), "hipMalloc(a0)");
    for (int l = 1; l < 4; ++l) CF_HIP(hipMalloc(&c->a[l], (size_t)P * 32 * 2), "hipMalloc(activations)");
    CF_HIP(hipMalloc(&c->resid, (size_t)P * 4 * 4), "hipMalloc(residual)");
    CF_HIP(hipMalloc(&c->dz3, (size_t)P * 8 * 2), "hipMalloc(dz)");
    CF_HIP(hipMalloc(&c->dzA, (size_t)P * 32 * 2), "hipMalloc(dz)");
    CF_HIP(hipMalloc(&c->dzB, (size_t)P * 32 * 2), "hipMalloc(dz)");
    c->cap_px = P;
    return LF_OK;
}

int pack(lf_corrector *c, hipStream_t s) {
    if (c->packed) return LF_OK;
    CF_HIP(corr_pack(c->prm, c->L, c->wbuf, c->bbuf, s), "pack weights");
    c->packed = true;
    return LF_OK;
}

// forward of all four layers into c->a[1..3] and c->resid
int forward(lf_corrector *c, const float *rgb, const float *wsum, const uint8_t *count, int32_t N, int32_t W,
            int32_t H, hipStream_t s) {
    const int64_t P = (int64_t)N * W * H;
    int rc = ensure_px(c, P);
    if (rc) return rc;
    rc = pack(c, s);
    if (rc) return rc;
    CF_HIP(corr_input(rgb, wsum, count, P, c->a[0], s), "corrector input");
    for (int l = 0; l < 4; ++l) {
        const CorrLayer &y = c->L.layer[l];
        void *out = l < 3 ? (void *)c->a[l + 1] : (void *)c->resid;
        CF_HIP(corr_conv(l, false, c->a[l], N, H, W, c->wbuf + y.wf_off, c->bbuf + y.b_off, out, nullptr, s),
               "corrector conv");
    }
    return LF_OK;
}

int check_images(const float *rgb, const float *wsum, const uint8_t *count, int32_t N, int32_t W, int32_t H) {
    if (!rgb || !wsum || !count) return cfail(LF_EINVAL, "rgb, wsum and count must not be NULL");
    if (N <= 0 || W <= 0 || H <= 0 || W > 32768 || H > 32768) return cfail(LF_EINVAL, "bad image batch %dx%dx%d", N, W, H);
    if ((int64_t)N * W * H > ((int64_t)1 << 31)) return cfail(LF_EINVAL, "image batch too large");
    return LF_OK;
}

}  // namespace

extern "C" {

int lf_corrector_create(const float *params, lf_corrector **out) {
    if (!out) return cfail(LF_EINVAL, "NULL argument");
    *out = nullptr;
    lf_corrector *c = new lf_corrector();
    auto bail = [&](int rc) {
        lf_corrector_free(c);
        return rc;
    };
    hipError_t e = hipSuccess;
    for (float **p : {&c->prm, &c->m1, &c->m2, &c->grad})
        if (e == hipSuccess) e = hipMalloc(p, sizeof(float) * kCorrParams);
    if (e == hipSuccess) e = hipMalloc(&c->wbuf, sizeof(uint16_t) * wbuf_elems(c->L));
    if (e == hipSuccess) e = hipMalloc(&c->bbuf, sizeof(float) * 128);
    if (e == hipSuccess) e = hipMalloc(&c->partial, sizeof(float) * kDwSlots * (9 * 32 * 32 + 32));
    if (e == hipSuccess) e = hipMalloc(&c->loss_part, sizeof(float) * kLossBlocks);
    if (e == hipSuccess) e = hipMemset(c->m1, 0, sizeof(float) * kCorrParams);
    if (e == hipSuccess) e = hipMemset(c->m2, 0, sizeof(float) * kCorrParams);
    if (e == hipSuccess) e = hipMemset(c->prm, 0, sizeof(float) * kCorrParams);
    if (e == hipSuccess && params)
        e = hipMemcpy(c->prm, params, sizeof(float) * kCorrParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        int dev = 0, n_cu = 0, per_cu = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = corr_fused_occupancy(&per_cu);
        c->fused_grid = std::max(1, n_cu * std::max(1, per_cu));
    }
    if (e != hipSuccess)
        return bail(cfail(e == hipErrorOutOfMemory ? LF_ENOMEM : LF_EHIP, "corrector create: %s", hipGetErrorString(e)));
    *out = c;
    return LF_OK;
}

int lf_corrector_set_params(lf_corrector *c, const float *params) {
    if (!c || !params) return cfail(LF_EINVAL, "NULL argument");
    CF_HIP(hipMemcpy(c->prm, params, sizeof(float) * kCorrParams, hipMemcpyHostToDevice), "set params");
    CF_HIP(hipMemset(c->m1, 0, sizeof(float) * kCorrParams), "reset optimiser");
    CF_HIP(hipMemset(c->m2, 0, sizeof(float) * kCorrParams), "reset optimiser");
    c->step = 0;
    c->packed = false;
    return LF_OK;
}

int lf_corrector_get_params(lf_corrector *c, float *params, int64_t *step) {
    if (!c || !params) return cfail(LF_EINVAL, "NULL argument");
    CF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    CF_HIP(hipMemcpy(params, c->prm, sizeof(float) * kCorrParams, hipMemcpyDeviceToHost), "get params");
    if (step) *step = c->step;
    return LF_OK;
}

int lf_corrector_get_state(lf_corrector *c, float *params, float *adam_m, float *adam_v, int64_t *step) {
    if (!c || !params || !adam_m || !adam_v || !step) return cfail(LF_EINVAL, "NULL argument");
    CF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    CF_HIP(hipMemcpy(params, c->prm, sizeof(float) * kCorrParams, hipMemcpyDeviceToHost), "get params");
    CF_HIP(hipMemcpy(adam_m, c->m1, sizeof(float) * kCorrParams, hipMemcpyDeviceToHost), "get first moments");
    CF_HIP(hipMemcpy(adam_v, c->m2, sizeof(float) * kCorrParams, hipMemcpyDeviceToHost), "get second moments");
    *step = c->step;
    return LF_OK;
}

int lf_corrector_set_state(lf_corrector *c, const float *params, const float *adam_m, const float *adam_v,
                           int64_t step) {
    if (!c || !params || !adam_m || !adam_v) return cfail(LF_EINVAL, "NULL argument");
    if (step < 0) return cfail(LF_EINVAL, "step must be >= 0 (got %lld)", (long long)step);
    for (int64_t k = 0; k < kCorrParams; ++k)
        if (!std::isfinite(params[k]) || !std::isfinite(adam_m[k]) || !(adam_v[k] >= 0.0f) || !std::isfinite(adam_v[k]))
            return cfail(LF_EINVAL, "state entry %lld is not finite (or a second moment is negative)", (long long)k);
    // renders and training steps already queued on any stream may still read the state
    CF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    CF_HIP(hipMemcpy(c->prm, params, sizeof(float) * kCorrParams, hipMemcpyHostToDevice), "set params");
    CF_HIP(hipMemcpy(c->m1, adam_m, sizeof(float) * kCorrParams, hipMemcpyHostToDevice), "set first moments");
    CF_HIP(hipMemcpy(c->m2, adam_v, sizeof(float) * kCorrParams, hipMemcpyHostToDevice), "set second moments");
    c->step = step;
    c->packed = false;
    return LF_OK;
}

int lf_corrector_apply(lf_corrector *c, const float *rgb, const float *wsum, const uint8_t *count, int32_t n_images,
                       int32_t W, int32_t H, float fallback_thresh, float *out_rgb, uint8_t *out_fallback,
                       float *out_resid, void *hip_stream) {
    // buffer arguments first (host-side checks only), then the handle
    int rc = check_images(rgb, wsum, count, n_images, W, H);
    if (rc) return rc;
    if (!out_rgb) return cfail(LF_EINVAL, "out_rgb must not be NULL");
    if (std::isnan(fallback_thresh) || fallback_thresh < 0.0f) return cfail(LF_EINVAL, "fallback_thresh must be >= 0");
    {
        // the fused kernel reads a halo around each tile and the next tile's
        // inputs while other workgroups write their outputs: outputs may not
        // overlap any input
        const int64_t P = (int64_t)n_images * W * H;
        const Span in[3] = {{rgb, P * 12}, {wsum, P * 4}, {count, P}};
        const Span out[3] = {{out_rgb, P * 12}, {out_fallback, P}, {out_resid, P * 12}};
        static const char *in_name[3] = {"rgb", "wsum", "count"};
        static const char *out_name[3] = {"out_rgb", "out_fallback", "out_resid"};
        for (int i = 0; i < 3; ++i)
            for (int o = 0; o < 3; ++o)
                if (overlaps(in[i], out[o]))
                    return cfail(LF_EINVAL, "%s overlaps %s: outputs must not share memory with inputs", out_name[o],
                                 in_name[i]);
        for (int o = 0; o < 3; ++o)
            for (int q = o + 1; q < 3; ++q)
                if (overlaps(out[o], out[q]))
                    return cfail(LF_EINVAL, "%s overlaps %s: outputs must be distinct", out_name[o], out_name[q]);
    }
    if (!c) return cfail(LF_EINVAL, "NULL corrector");
    hipStream_t s = (hipStream_t)hip_stream;
    rc = pack(c, s);
    if (rc) return rc;
    const int grid = std::min(c->fused_grid, corr_fused_tiles(n_images, H, W));
    CF_HIP(corr_fused(rgb, wsum, count, n_images, H, W, c->wbuf, c->bbuf, c->L, fallback_thresh, out_rgb, out_fallback,
                      out_resid, grid, s),
           "corrector inference");
    return LF_OK;
}

int lf_corrector_train_step(lf_corrector *c, const float *rgb, const float *wsum, const uint8_t *count,
                            const float *ref, int32_t n_images, int32_t W, int32_t H, float lr, float *loss_out,
                            float *grad_out, void *hip_stream) {
    if (!c) return cfail(LF_EINVAL, "NULL corrector");
    int rc = check_images(rgb, wsum, count, n_images, W, H);
    if (rc) return rc;
    if (!ref) return cfail(LF_EINVAL, "ref must not be NULL");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return cfail(LF_EINVAL, "lr must be finite and >= 0");
    hipStream_t s = (hipStream_t)hip_stream;
    rc = forward(c, rgb, wsum, count, n_images, W, H, s);
    if (rc) return rc;
    const int64_t P = (int64_t)n_images * W * H;
    CF_HIP(corr_loss(rgb, c->resid, ref, P, c->dz3, c->loss_part, kLossBlocks, s), "corrector loss");
    // backward: layer 3 (no ReLU) down to layer 0
    const uint16_t *dz = c->dz3;
    uint16_t *next[2] = {c->dzA, c->dzB};
    for (int l = 3; l >= 0; --l) {
        const CorrLayer &y = c->L.layer[l];
        const int len = 9 * y.cin * y.cout + y.cout;
        CF_HIP(corr_dw(l, c->a[l], dz, n_images, H, W, y.cin, y.cout, c->partial, kDwSlots, s), "corrector dW");
        CF_HIP(corr_reduce(c->partial, kDwSlots, len, c->grad + y.poff, s), "corrector dW reduce");
        if (l > 0) {
            uint16_t *o = next[l & 1];
            CF_HIP(corr_conv(l, true, dz, n_images, H, W, c->wbuf + y.wb_off, nullptr, o, c->a[l], s),
                   "corrector dX");
            dz = o;
        }
    }
    if (lr > 0.0f) {
        c->step += 1;
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)c->step)));
        const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)c->step)));
        CF_HIP(corr_adam(c->prm, c->grad, c->m1, c->m2, kCorrParams, lr, b1, b2, eps, c1, c2, s), "adam");
        c->packed = false;
    }
    if (loss_out || grad_out) {
        CF_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (loss_out) {
            std::vector<float> lp(kLossBlocks);
            CF_HIP(hipMemcpy(lp.data(), c->loss_part, sizeof(float) * kLossBlocks, hipMemcpyDeviceToHost), "read loss");
            double acc = 0.0;
            for (float v : lp) acc += v;
            *loss_out = (float)(acc / (3.0 * (double)P));
        }
        if (grad_out)
            CF_HIP(hipMemcpy(grad_out, c->grad, sizeof(float) * kCorrParams, hipMemcpyDeviceToHost), "read grad");
    }
    return LF_OK;
}

void lf_corrector_free(lf_corrector *c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    for (void *p : {(void *)c->prm, (void *)c->m1, (void *)c->m2, (void *)c->grad, (void *)c->wbuf, (void *)c->bbuf,
                    (void *)c->partial, (void *)c->loss_part, (void *)c->resid, (void *)c->dz3, (void *)c->dzA,
                    (void *)c->dzB, (void *)c->a[0], (void *)c->a[1], (void *)c->a[2], (void *)c->a[3]})
        if (p) (void)hipFree(p);
    delete c;
}

}  // extern "C"
