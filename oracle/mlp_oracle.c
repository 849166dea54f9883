/*
 * mlp_oracle.c -- FP64 CPU reference of the seeding network (test
 * infrastructure only; shares no code with the GPU kernels).
 *
 * Network: x (n_in) -> Linear(n_in, H) -> GELU -> Linear(H, H) -> GELU ->
 * Linear(H, n_out).  GELU is the exact form 0.5 z (1 + erf(z / sqrt 2)).
 * Weights are row-major W[out][in]; biases b[out].
 *
 * Loss over a batch of B rows with targets t_i (n_out - 1 values) and a in {0, 1}:
 *   L = (1/B) sum_i [ a_i sum_{o < n_out-1} (y_io - t_io)^2 + BCE(y_i,n_out-1, a_i) ],
 *   BCE(z, a) = max(z, 0) - z a + log(1 + exp(-|z|)).
 * The first outputs are the predicted local parameters (u for a curve piece,
 * (u, v) for a surface patch), the last one the logit of "the projection lies
 * on this piece"; the parameter loss is masked by a (MSE * accept + BCE).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double ml_gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }
static double ml_dgelu(double z)
{
    return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
}

/* Forward and (optionally) backward for one batch.  params holds W1 (H x n_in),
 * b1 (H), W2 (H x H), b2 (H), W3 (n_out x H), b3 (n_out) back to back; grad
 * (nullable) receives dL/dparams in the same layout; y (nullable) receives the
 * outputs [B x n_out]; target [B x (n_out - 1)] and accept [B] (nullable
 * together: forward only).  Returns the loss. */
double orc_mlp_loss(int n_in, int H, int n_out, const double *params, int64_t B, const double *x,
                    const double *target, const double *accept, double *y, double *grad)
{
    const double *W1 = params, *b1 = W1 + (size_t)H * n_in, *W2 = b1 + H, *b2 = W2 + (size_t)H * H,
                 *W3 = b2 + H, *b3 = W3 + (size_t)n_out * H;
    size_t np = (size_t)H * n_in + H + (size_t)H * H + H + (size_t)n_out * H + n_out;
    if (grad) memset(grad, 0, sizeof(double) * np);
    double *gW1 = grad, *gb1 = grad ? gW1 + (size_t)H * n_in : NULL, *gW2 = grad ? gb1 + H : NULL,
           *gb2 = grad ? gW2 + (size_t)H * H : NULL, *gW3 = grad ? gb2 + H : NULL,
           *gb3 = grad ? gW3 + (size_t)n_out * H : NULL;
    double *z1 = (double *)malloc(sizeof(double) * H), *h1 = (double *)malloc(sizeof(double) * H);
    double *z2 = (double *)malloc(sizeof(double) * H), *h2 = (double *)malloc(sizeof(double) * H);
    double *d2 = (double *)malloc(sizeof(double) * H), *d1 = (double *)malloc(sizeof(double) * H);
    double out[16], dout[16];
    double loss = 0.0;
    for (int64_t r = 0; r < B; ++r) {
        const double *xr = x + (size_t)r * n_in;
        for (int j = 0; j < H; ++j) {
            double s = b1[j];
            for (int k = 0; k < n_in; ++k) s += W1[(size_t)j * n_in + k] * xr[k];
            z1[j] = s;
            h1[j] = ml_gelu(s);
        }
        for (int j = 0; j < H; ++j) {
            double s = b2[j];
            for (int k = 0; k < H; ++k) s += W2[(size_t)j * H + k] * h1[k];
            z2[j] = s;
            h2[j] = ml_gelu(s);
        }
        for (int o = 0; o < n_out; ++o) {
            double s = b3[o];
            for (int k = 0; k < H; ++k) s += W3[(size_t)o * H + k] * h2[k];
            out[o] = s;
            if (y) y[(size_t)r * n_out + o] = s;
        }
        if (!target) continue;
        const double a = accept[r];
        const double z = out[n_out - 1];
        double mse = 0.0;
        for (int o = 0; o < n_out - 1; ++o) {
            const double du = out[o] - target[(size_t)r * (n_out - 1) + o];
            mse += du * du;
            dout[o] = 2.0 * a * du / (double)B;
        }
        loss += a * mse + (z > 0 ? z : 0.0) - z * a + log1p(exp(-fabs(z)));
        if (!grad) continue;
        dout[n_out - 1] = (1.0 / (1.0 + exp(-z)) - a) / (double)B;
        for (int o = 0; o < n_out; ++o) {
            gb3[o] += dout[o];
            for (int k = 0; k < H; ++k) gW3[(size_t)o * H + k] += dout[o] * h2[k];
        }
        for (int k = 0; k < H; ++k) {
            double s = 0.0;
            for (int o = 0; o < n_out; ++o) s += dout[o] * W3[(size_t)o * H + k];
            d2[k] = s * ml_dgelu(z2[k]);
        }
        for (int j = 0; j < H; ++j) {
            gb2[j] += d2[j];
            for (int k = 0; k < H; ++k) gW2[(size_t)j * H + k] += d2[j] * h1[k];
        }
        for (int k = 0; k < H; ++k) {
            double s = 0.0;
            for (int j = 0; j < H; ++j) s += d2[j] * W2[(size_t)j * H + k];
            d1[k] = s * ml_dgelu(z1[k]);
        }
        for (int j = 0; j < H; ++j) {
            gb1[j] += d1[j];
            for (int k = 0; k < n_in; ++k) gW1[(size_t)j * n_in + k] += d1[j] * xr[k];
        }
    }
    free(z1); free(h1); free(z2); free(h2); free(d2); free(d1);
    return loss / (double)(B > 0 ? B : 1);
}
