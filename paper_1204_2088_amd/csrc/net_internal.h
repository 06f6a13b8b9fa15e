// net_internal.h -- launchers of the warm-start network kernels (net_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace hsf {

constexpr int kNetMaxWidth = 32;   // widest layer the weight-gradient kernel supports

// Input of a convolution, composed while its tile is staged (never stored):
//   CONV_IN_PLAIN  x1                    (x1 on the convolution's box)
//   CONV_IN_ADD    x1 + x2               (both on the convolution's box)
//   CONV_IN_UP     nearest 2x upsampling of x1 (x1 on the box of half the edge)
//   CONV_IN_POOL   2x2x2 average of x1   (x1 on the box of twice the edge)
//   CONV_IN_PACKED xp                    (forward only)
// x1, x2 are FP32 [batch][ci][site] on their own boxes; xp is BF16 [batch][site][cip]
// (cip = ci rounded up to 8, channels ci..cip-1 zero), the layout the forward
// convolution stages its tile in.  A plain input may carry a per-channel affine map,
// applied as (x - shift[c]) scale[c] while staging (forward only).
enum { CONV_IN_PLAIN = 0, CONV_IN_ADD = 1, CONV_IN_UP = 2, CONV_IN_POOL = 3, CONV_IN_PACKED = 4 };
struct ConvIn {
    const float *x1 = nullptr, *x2 = nullptr;
    int mode = CONV_IN_PLAIN;
    const __bf16 *xp = nullptr;
    const float *shift = nullptr, *scale = nullptr;
};

// Outputs of a forward convolution (any may be null):
//   Y   FP32 [batch][co][site]  acc + bias, then (. - shift[o]) scale[o] if shift is set
//   A   FP32 [batch][co][site]  silu(acc + bias)
//   Ap  BF16 [batch][site][cp]  silu(acc + bias) rounded to BF16, cp = co rounded up to
//       8, channels co..cp-1 written as zero (the CONV_IN_PACKED input of the next layer)
struct ConvOut {
    float *Y = nullptr, *A = nullptr;
    __bf16 *Ap = nullptr;
    const float *shift = nullptr, *scale = nullptr;
};

void net_conv_fwd(hipStream_t s, ConvIn in, int B, int ci, int cip, const __bf16 *Wm, int kp, int co, int cop,
                  const float *bias, ConvOut out, int L);
int net_wgrad_slices(int B, int L, int cop, int kp);
void net_conv_wgrad(hipStream_t s, ConvIn in, int B, int ci, int cip, const float *dY, int co, int cop, int kp,
                    int L, float *part, float *dWm);
void net_silu_bwd(hipStream_t s, const float *dA, const float *Y, float *dY, long long n);
void net_pool_bwd(hipStream_t s, const float *dout, float *din, int L, long long n_in, int add);
void net_up_bwd(hipStream_t s, const float *dout, float *din, int L, long long n_in, int add);
void net_accum(hipStream_t s, float *dst, const float *src, long long n, int add);
int net_channel_parts(int C);
void net_channel_sum(hipStream_t s, const float *g, int B, int C, long long V, double *part, float *out);
int net_mse(hipStream_t s, const float *p, const float *t, float *dp, long long n, float inv_count, double *part);
void net_adam(hipStream_t s, float *w, const float *g, float *m, float *v, long long n, float lr, float b1, float b2,
              float eps, float c1, float c2);
void net_stage_weights(hipStream_t s, const float *W, int co, int ci, int cip, int kp, int cop_rows, __bf16 *Wm,
                       int cip_t, int kp_t, int cop_rows_t, __bf16 *Wt);
void net_unstage_grad(hipStream_t s, const float *dWm, int co, int ci, int cip, int kp, float *dW);
// Warm start from the network.  mode 0: input phi; 1: (h0, (phi - h0) / rms);
// 2: (h0, (phi - 2 h0 + h1) / rms), rms computed on the device into *rms.
void net_warm_input(hipStream_t s, const double *phi, const double *h0, const double *h1, int nsp, long long V,
                    int mode, double *part, int max_parts, double *rms, float *x);
void net_warm_apply(hipStream_t s, double *w, const float *p, long long V, int mode, const double *rms,
                    const double *wh0, const double *wh1);
void net_shift_fields(hipStream_t s, double *w, const double *wh0, const double *wh1, long long n);
void net_affine(hipStream_t s, float *x, int C, long long V, long long n, const float *shift, const float *scale);
// A training sample of one replica from three (phi, w) states in the field layout (nsp x V
// doubles): x = (phi0, delta phi / r) as the warm start feeds the network, y = delta w / r
// over the polymer channels, r = rms of delta phi (written to rms[0]); mode 1: delta =
// new - 0, mode 2: new - 2 * 0 + 1.
void net_sample(hipStream_t s, const double *phi, const double *phi0, const double *phi1, const double *w,
                const double *w0, const double *w1, int nsp, long long V, int mode, double *part, int max_parts,
                double *rms, float *x, float *y);
// Mean and root mean square per channel of x [batch][C][V] into out[2 C] (device);
// part holds 2 C nblk doubles.
void net_channel_moments(hipStream_t s, const float *x, int batch, int C, long long V, double *part, int nblk,
                         double *out);

}  // namespace hsf
