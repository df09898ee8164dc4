/*
 * FP64 CPU oracle of the residual corrector's layers (test infrastructure
 * only; shares nothing with the HIP kernels).
 *
 * One layer: y = act(z), z[n][p][co] = b[co] + sum_{ky,kx in 0..2} sum_ci
 * x[n][py+ky-1][px+kx-1][ci] * w[ky][kx][ci][co] (cross-correlation, zero
 * padding outside the image, NHWC activations), act = ReLU or identity.
 * The backward pass takes dL/dy and returns dL/dx, dL/dw, dL/db by the chain
 * rule written out as plain loops.
 */
#include <stdint.h>
#include <string.h>

void orc_conv3x3_fwd(const double *x, int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout,
                     const double *w, const double *b, double *y, int32_t relu) {
    for (int32_t n = 0; n < N; ++n)
        for (int32_t py = 0; py < H; ++py)
            for (int32_t px = 0; px < W; ++px) {
                double *yo = y + (((int64_t)n * H + py) * W + px) * Cout;
                for (int32_t co = 0; co < Cout; ++co) {
                    double z = b[co];
                    for (int32_t ky = 0; ky < 3; ++ky) {
                        const int32_t sy = py + ky - 1;
                        if (sy < 0 || sy >= H) continue;
                        for (int32_t kx = 0; kx < 3; ++kx) {
                            const int32_t sx = px + kx - 1;
                            if (sx < 0 || sx >= W) continue;
                            const double *xi = x + (((int64_t)n * H + sy) * W + sx) * Cin;
                            const double *wk = w + ((int64_t)(ky * 3 + kx) * Cin) * Cout + co;
                            for (int32_t ci = 0; ci < Cin; ++ci) z += xi[ci] * wk[(int64_t)ci * Cout];
                        }
                    }
                    yo[co] = (relu && z < 0.0) ? 0.0 : z;
                }
            }
}

/* dy = dL/dy; y = the layer's output (for the ReLU mask). dx may be NULL. */
void orc_conv3x3_bwd(const double *x, const double *y, int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout,
                     const double *w, const double *dy, double *dx, double *dw, double *db, int32_t relu) {
    if (dx) memset(dx, 0, sizeof(double) * (size_t)N * H * W * Cin);
    memset(dw, 0, sizeof(double) * 9 * (size_t)Cin * Cout);
    memset(db, 0, sizeof(double) * (size_t)Cout);
    for (int32_t n = 0; n < N; ++n)
        for (int32_t py = 0; py < H; ++py)
            for (int32_t px = 0; px < W; ++px) {
                const int64_t o = (((int64_t)n * H + py) * W + px) * Cout;
                for (int32_t co = 0; co < Cout; ++co) {
                    double dz = dy[o + co];
                    if (relu && !(y[o + co] > 0.0)) dz = 0.0;
                    if (dz == 0.0) continue;
                    db[co] += dz;
                    for (int32_t ky = 0; ky < 3; ++ky) {
                        const int32_t sy = py + ky - 1;
                        if (sy < 0 || sy >= H) continue;
                        for (int32_t kx = 0; kx < 3; ++kx) {
                            const int32_t sx = px + kx - 1;
                            if (sx < 0 || sx >= W) continue;
                            const int64_t xi = (((int64_t)n * H + sy) * W + sx) * Cin;
                            const int64_t wk = ((int64_t)(ky * 3 + kx) * Cin) * Cout + co;
                            for (int32_t ci = 0; ci < Cin; ++ci) {
                                dw[wk + (int64_t)ci * Cout] += x[xi + ci] * dz;
                                if (dx) dx[xi + ci] += w[wk + (int64_t)ci * Cout] * dz;
                            }
                        }
                    }
                }
            }
}
