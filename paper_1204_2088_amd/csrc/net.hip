// net.hip -- the warm-start network (a build addition to the method): a 4-level
// U-Net on the periodic lattice that maps the densities (phi_A, phi_B[, phi_S])
// to the polymer fields (w_A, w_B), trained on (phi, w) pairs produced by the
// inversion itself.  Forward and backward passes run in the kernels of
// net_kernels.hip (convolutions on the BF16 matrix cores, FP32 accumulation);
// master weights and Adam moments are FP32.
//
// Topology (widths w1..w4, SiLU after every convolution except the last):
//   e1 = c(c(x, in->w1), w1->w1)                        level L
//   e2 = c(c(pool e1, w1->w2), w2->w2)                  level L/2
//   e3 = c(c(pool e2, w2->w3), w3->w3)                  level L/4
//   e4 = c(c(pool e3, w3->w4), w4->w4)                  level L/8
//   d3 = c(c(up e4, w4->w3) + e3, w3->w3)               level L/4
//   d2 = c(c(up d3, w3->w2) + e2, w2->w2)               level L/2
//   d1 = c(c(up d2, w2->w1) + e1, w1->w1)               level L
//   out = conv(d1, w1->out)                             level L (no activation)
// c(.) = SiLU(3x3x3 periodic convolution + bias); pool = 2x2x2 average; up = nearest.
// Parameter vector: for layers 0..14 in this order, W[co][ci][27] then b[co].
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "hsf.h"
#include "net_internal.h"

using namespace hsf;

namespace {

constexpr int kLayers = 15;

int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct Layer {
    int ci, co, act, level;          // level 0..3 (box L >> level)
    int cip, kp, cop;                // forward matrix-core layout
    int cip_t, kp_t, cop_t;          // transposed-flipped layout (data gradient)
    long long w_off, b_off;          // offsets in the parameter vector
    __bf16 *Wm = nullptr, *Wt = nullptr;
    float *dWm = nullptr;            // weight gradient, matrix-core layout
};

struct Tensor {
    float *p = nullptr;
    int c = 0, level = 0;
};

}  // namespace

struct hsf_net {
    int in_ch = 0, out_ch = 0, w[4] = {0, 0, 0, 0};
    Layer layer[kLayers];
    long long n_params = 0;
    float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    float *norm = nullptr;           // device: input shift[in_ch], scale[in_ch]
    long long adam_t = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<void *> allocs;      // parameter-sized and weight buffers
    // activation buffers for the current (batch, box)
    int cur_B = 0, cur_L = 0;
    std::vector<void *> act_allocs;
    Tensor x0, y[kLayers], a[kLayers], p1, p2, p3, u3, u2, u1, t3, t2, t1;
    Tensor dy[kLayers], da[kLayers], dp1, dp2, dp3, du3, du2, du1, dt3, dt2, dt1, dout;
    float *target = nullptr, *wpart = nullptr;
    double *bpart = nullptr;         // per-channel partial sums of the bias gradient
    double *loss_part = nullptr, *loss_host = nullptr;
    int weights_staged = 0;
    int training = 0;                // the current forward pass feeds a backward pass
};

namespace {

int nfail(hsf_net *n, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (n) n->err = buf;
    return code;
}

#define NCHK(n, expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return nfail((n), HSF_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int nalloc(hsf_net *n, std::vector<void *> &list, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return nfail(n, HSF_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    list.push_back(*p);
    return HSF_OK;
}

long long vol(int L, int level)
{
    const long long l = L >> level;
    return l * l * l;
}

void free_acts(hsf_net *n)
{
    for (void *p : n->act_allocs) (void)hipFree(p);
    n->act_allocs.clear();
    n->cur_B = n->cur_L = 0;
    // forget every pointer into the freed buffers (a later allocation without the
    // gradient tensors must not find stale ones)
    for (Tensor *t : {&n->x0, &n->p1, &n->p2, &n->p3, &n->u3, &n->u2, &n->u1, &n->t3, &n->t2, &n->t1, &n->dp1,
                      &n->dp2, &n->dp3, &n->du3, &n->du2, &n->du1, &n->dt3, &n->dt2, &n->dt1, &n->dout})
        *t = Tensor();
    for (int l = 0; l < kLayers; ++l) n->y[l] = n->a[l] = n->dy[l] = n->da[l] = Tensor();
    n->target = n->wpart = nullptr;
    n->bpart = nullptr;
    n->loss_part = nullptr;
}

// (Re)allocate the activation and gradient tensors for batch B on an L^3 box.
int ensure_acts(hsf_net *n, int B, int L, bool grads)
{
    if (n->cur_B == B && n->cur_L == L && (!grads || n->dout.p)) return HSF_OK;
    free_acts(n);
    int rc = HSF_OK;
    auto T = [&](Tensor &t, int c, int level) {
        t.c = c;
        t.level = level;
        if (rc == HSF_OK) rc = nalloc(n, n->act_allocs, (void **)&t.p, sizeof(float) * (size_t)B * c * vol(L, level));
    };
    const int *w = n->w;
    T(n->x0, n->in_ch, 0);
    for (int l = 0; l < kLayers; ++l) {
        T(n->y[l], n->layer[l].co, n->layer[l].level);
        if (n->layer[l].act) T(n->a[l], n->layer[l].co, n->layer[l].level);
    }
    T(n->p1, w[0], 1);
    T(n->p2, w[1], 2);
    T(n->p3, w[2], 3);
    T(n->u3, w[3], 2);
    T(n->u2, w[2], 1);
    T(n->u1, w[1], 0);
    T(n->t3, w[2], 2);
    T(n->t2, w[1], 1);
    T(n->t1, w[0], 0);
    if (grads) {
        for (int l = 0; l < kLayers; ++l) {
            T(n->dy[l], n->layer[l].co, n->layer[l].level);
            T(n->da[l], n->layer[l].co, n->layer[l].level);
        }
        T(n->dp1, w[0], 1);
        T(n->dp2, w[1], 2);
        T(n->dp3, w[2], 3);
        T(n->du3, w[3], 2);
        T(n->du2, w[2], 1);
        T(n->du1, w[1], 0);
        T(n->dt3, w[2], 2);
        T(n->dt2, w[1], 1);
        T(n->dt1, w[0], 0);
        T(n->dout, n->out_ch, 0);
        if (rc == HSF_OK)
            rc = nalloc(n, n->act_allocs, (void **)&n->target, sizeof(float) * (size_t)B * n->out_ch * vol(L, 0));
        size_t wp = 0;
        for (int l = 0; l < kLayers; ++l) {
            const Layer &Ly = n->layer[l];
            wp = std::max(wp, (size_t)net_wgrad_slices(B, L >> Ly.level, Ly.cop, Ly.kp) * Ly.cop * Ly.kp);
        }
        if (rc == HSF_OK) rc = nalloc(n, n->act_allocs, (void **)&n->wpart, sizeof(float) * wp);
        if (rc == HSF_OK)
            rc = nalloc(n, n->act_allocs, (void **)&n->bpart, sizeof(double) * net_channel_parts(kNetMaxWidth));
        const size_t lb = ((size_t)B * n->out_ch * vol(L, 0) + 255) / 256;
        if (rc == HSF_OK) rc = nalloc(n, n->act_allocs, (void **)&n->loss_part, sizeof(double) * lb);
    }
    if (rc != HSF_OK) {
        free_acts(n);
        return rc;
    }
    n->cur_B = B;
    n->cur_L = L;
    return HSF_OK;
}

int stage_weights(hsf_net *n)
{
    for (int l = 0; l < kLayers; ++l) {
        const Layer &Ly = n->layer[l];
        net_stage_weights(n->stream, n->params + Ly.w_off, Ly.co, Ly.ci, Ly.cip, Ly.kp, Ly.cop, Ly.Wm, Ly.cip_t,
                          Ly.kp_t, Ly.cop_t, Ly.Wt);
    }
    NCHK(n, hipGetLastError());
    n->weights_staged = 1;
    return HSF_OK;
}

// Forward of layer l.  The pre-activation y[l] is kept only when a backward pass
// follows (training); inference writes the activation alone.
void conv(hsf_net *n, int l, const Tensor &in, int B)
{
    const Layer &Ly = n->layer[l];
    float *y = (Ly.act && !n->training) ? nullptr : n->y[l].p;
    net_conv_fwd(n->stream, in.p, B, Ly.ci, Ly.cip, Ly.Wm, Ly.kp, Ly.co, Ly.cop, n->params + Ly.b_off, y,
                 Ly.act ? n->a[l].p : nullptr, n->cur_L >> Ly.level);
}

long long numel(const hsf_net *n, const Tensor &t) { return (long long)n->cur_B * t.c * vol(n->cur_L, t.level); }

void forward(hsf_net *n)
{
    const int B = n->cur_B, L = n->cur_L;
    hipStream_t s = n->stream;
    net_affine(s, n->x0.p, n->in_ch, vol(L, 0), numel(n, n->x0), n->norm, n->norm + n->in_ch);
    conv(n, 0, n->x0, B);
    conv(n, 1, n->a[0], B);                                   // e1 = a[1]
    net_pool(s, n->a[1].p, n->p1.p, L, numel(n, n->p1));
    conv(n, 2, n->p1, B);
    conv(n, 3, n->a[2], B);                                   // e2 = a[3]
    net_pool(s, n->a[3].p, n->p2.p, L >> 1, numel(n, n->p2));
    conv(n, 4, n->p2, B);
    conv(n, 5, n->a[4], B);                                   // e3 = a[5]
    net_pool(s, n->a[5].p, n->p3.p, L >> 2, numel(n, n->p3));
    conv(n, 6, n->p3, B);
    conv(n, 7, n->a[6], B);                                   // e4 = a[7]
    net_up(s, n->a[7].p, n->u3.p, L >> 2, numel(n, n->u3));
    conv(n, 8, n->u3, B);
    net_add(s, n->a[8].p, n->a[5].p, n->t3.p, numel(n, n->t3));
    conv(n, 9, n->t3, B);                                     // d3 = a[9]
    net_up(s, n->a[9].p, n->u2.p, L >> 1, numel(n, n->u2));
    conv(n, 10, n->u2, B);
    net_add(s, n->a[10].p, n->a[3].p, n->t2.p, numel(n, n->t2));
    conv(n, 11, n->t2, B);                                    // d2 = a[11]
    net_up(s, n->a[11].p, n->u1.p, L, numel(n, n->u1));
    conv(n, 12, n->u1, B);
    net_add(s, n->a[12].p, n->a[1].p, n->t1.p, numel(n, n->t1));
    conv(n, 13, n->t1, B);                                    // d1 = a[13]
    conv(n, 14, n->a[13], B);                                 // out = y[14]
}

// Gradient of layer l given dy[l]: weight and bias gradients, and (din != null) the
// gradient of its input.
void conv_bwd(hsf_net *n, int l, const Tensor &in, float *din)
{
    const Layer &Ly = n->layer[l];
    const int B = n->cur_B, Ll = n->cur_L >> Ly.level;
    net_conv_wgrad(n->stream, in.p, B, Ly.ci, Ly.cip, n->dy[l].p, Ly.co, Ly.cop, Ly.kp, Ll, n->wpart, Ly.dWm);
    net_unstage_grad(n->stream, Ly.dWm, Ly.co, Ly.ci, Ly.cip, Ly.kp, n->grad + Ly.w_off);
    net_channel_sum(n->stream, n->dy[l].p, B, Ly.co, vol(n->cur_L, Ly.level), n->bpart, n->grad + Ly.b_off);
    if (din)
        net_conv_fwd(n->stream, n->dy[l].p, B, Ly.co, Ly.cip_t, Ly.Wt, Ly.kp_t, Ly.ci, Ly.cop_t, nullptr, din,
                     nullptr, Ll);
}

// dy[l] = dA * silu'(y[l])
void act_bwd(hsf_net *n, int l, const float *dA)
{
    net_silu_bwd(n->stream, dA, n->y[l].p, n->dy[l].p, numel(n, n->y[l]));
}

void backward(hsf_net *n)
{
    hipStream_t s = n->stream;
    const int L = n->cur_L;
    // out = y[14] = conv(d1): dy[14] = dout
    (void)hipMemcpyAsync(n->dy[14].p, n->dout.p, sizeof(float) * numel(n, n->dout), hipMemcpyDeviceToDevice, s);
    conv_bwd(n, 14, n->a[13], n->da[13].p);
    act_bwd(n, 13, n->da[13].p);
    conv_bwd(n, 13, n->t1, n->dt1.p);                         // t1 = a[12] + e1
    act_bwd(n, 12, n->dt1.p);
    conv_bwd(n, 12, n->u1, n->du1.p);
    net_up_bwd(s, n->du1.p, n->da[11].p, L, numel(n, n->a[11]));
    act_bwd(n, 11, n->da[11].p);
    conv_bwd(n, 11, n->t2, n->dt2.p);                         // t2 = a[10] + e2
    act_bwd(n, 10, n->dt2.p);
    conv_bwd(n, 10, n->u2, n->du2.p);
    net_up_bwd(s, n->du2.p, n->da[9].p, L >> 1, numel(n, n->a[9]));
    act_bwd(n, 9, n->da[9].p);
    conv_bwd(n, 9, n->t3, n->dt3.p);                          // t3 = a[8] + e3
    act_bwd(n, 8, n->dt3.p);
    conv_bwd(n, 8, n->u3, n->du3.p);
    net_up_bwd(s, n->du3.p, n->da[7].p, L >> 2, numel(n, n->a[7]));   // e4
    act_bwd(n, 7, n->da[7].p);
    conv_bwd(n, 7, n->a[6], n->da[6].p);
    act_bwd(n, 6, n->da[6].p);
    conv_bwd(n, 6, n->p3, n->dp3.p);
    // e3 = a[5] feeds the pooling and the skip sum t3
    net_pool_bwd(s, n->dp3.p, n->da[5].p, L >> 2, numel(n, n->a[5]), 0);
    net_add(s, n->dt3.p, nullptr, n->da[5].p, numel(n, n->a[5]));
    act_bwd(n, 5, n->da[5].p);
    conv_bwd(n, 5, n->a[4], n->da[4].p);
    act_bwd(n, 4, n->da[4].p);
    conv_bwd(n, 4, n->p2, n->dp2.p);
    net_pool_bwd(s, n->dp2.p, n->da[3].p, L >> 1, numel(n, n->a[3]), 0);   // e2
    net_add(s, n->dt2.p, nullptr, n->da[3].p, numel(n, n->a[3]));
    act_bwd(n, 3, n->da[3].p);
    conv_bwd(n, 3, n->a[2], n->da[2].p);
    act_bwd(n, 2, n->da[2].p);
    conv_bwd(n, 2, n->p1, n->dp1.p);
    net_pool_bwd(s, n->dp1.p, n->da[1].p, L, numel(n, n->a[1]), 0);        // e1
    net_add(s, n->dt1.p, nullptr, n->da[1].p, numel(n, n->a[1]));
    act_bwd(n, 1, n->da[1].p);
    conv_bwd(n, 1, n->a[0], n->da[0].p);
    act_bwd(n, 0, n->da[0].p);
    conv_bwd(n, 0, n->x0, nullptr);
}

int copy_f32(hsf_net *n, float *dst, const float *src, size_t count, int where, hipMemcpyKind host_kind)
{
    if (!src || !dst) return nfail(n, HSF_EINVAL, "null pointer");
    if (where == HSF_DEVICE) {
        NCHK(n, hipMemcpyAsync(dst, src, count * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    } else if (where == HSF_HOST) {
        NCHK(n, hipMemcpyAsync(dst, src, count * sizeof(float), host_kind, n->stream));
        NCHK(n, hipStreamSynchronize(n->stream));
    } else {
        return nfail(n, HSF_EINVAL, "bad memory location");
    }
    return HSF_OK;
}

int check_box(hsf_net *n, int B, int L)
{
    if (B < 1 || L < 8 || (L % 8) != 0) return nfail(n, HSF_EINVAL, "batch %d, box %d: need L a multiple of 8", B, L);
    return HSF_OK;
}

// Loss (mean square error over batch, channels and sites) and gradients for the
// current inputs x0 and target.
int loss_and_grad(hsf_net *n, double *loss)
{
    if (!n->weights_staged) {
        int rc = stage_weights(n);
        if (rc) return rc;
    }
    n->training = 1;
    forward(n);
    n->training = 0;
    const long long cnt = numel(n, n->dout);
    const int blocks = net_mse(n->stream, n->y[14].p, n->target, n->dout.p, cnt, 1.0f / (float)cnt, n->loss_part);
    backward(n);
    NCHK(n, hipGetLastError());
    std::vector<double> lp(blocks);
    NCHK(n, hipMemcpyAsync(lp.data(), n->loss_part, sizeof(double) * blocks, hipMemcpyDeviceToHost, n->stream));
    NCHK(n, hipStreamSynchronize(n->stream));
    double s = 0.0;
    for (double v : lp) s += v;
    if (loss) *loss = s / (double)cnt;
    return HSF_OK;
}

// Deterministic parameter initialisation: uniform(-a, a) with a = sqrt(3 / fan_in)
// (a quarter of that for the output layer) from a splitmix64 hash of (seed, index);
// biases zero.
double unit_hash(unsigned long long seed, unsigned long long i)
{
    unsigned long long z = seed + 0x9E3779B97F4A7C15ULL * (i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

extern "C" {

int hsf_net_create(int in_ch, int out_ch, const int widths[4], unsigned long long seed, hsf_net **out)
{
    if (!out || !widths || in_ch < 1 || in_ch > kNetMaxWidth || out_ch < 1 || out_ch > kNetMaxWidth)
        return HSF_EINVAL;
    *out = nullptr;
    for (int i = 0; i < 4; ++i)
        if (widths[i] < 1 || widths[i] > kNetMaxWidth) return HSF_EINVAL;
    hsf_net *n = new hsf_net();
    n->in_ch = in_ch;
    n->out_ch = out_ch;
    for (int i = 0; i < 4; ++i) n->w[i] = widths[i];
    const int *w = widths;
    const int spec[kLayers][4] = {  // ci, co, act, level
        {in_ch, w[0], 1, 0}, {w[0], w[0], 1, 0}, {w[0], w[1], 1, 1}, {w[1], w[1], 1, 1},
        {w[1], w[2], 1, 2},  {w[2], w[2], 1, 2}, {w[2], w[3], 1, 3}, {w[3], w[3], 1, 3},
        {w[3], w[2], 1, 2},  {w[2], w[2], 1, 2}, {w[2], w[1], 1, 1}, {w[1], w[1], 1, 1},
        {w[1], w[0], 1, 0},  {w[0], w[0], 1, 0}, {w[0], out_ch, 0, 0}};
    long long off = 0;
    for (int l = 0; l < kLayers; ++l) {
        Layer &Ly = n->layer[l];
        Ly.ci = spec[l][0];
        Ly.co = spec[l][1];
        Ly.act = spec[l][2];
        Ly.level = spec[l][3];
        Ly.cip = round_up(Ly.ci, 8);
        Ly.kp = round_up(27 * Ly.cip, 32);
        Ly.cop = round_up(Ly.co, 16);
        Ly.cip_t = round_up(Ly.co, 8);
        Ly.kp_t = round_up(27 * Ly.cip_t, 32);
        Ly.cop_t = round_up(Ly.ci, 16);
        Ly.w_off = off;
        off += (long long)Ly.co * Ly.ci * 27;
        Ly.b_off = off;
        off += Ly.co;
    }
    n->n_params = off;
    int rc = HSF_OK;
    rc = nalloc(n, n->allocs, (void **)&n->params, sizeof(float) * off);
    if (rc == HSF_OK) rc = nalloc(n, n->allocs, (void **)&n->grad, sizeof(float) * off);
    if (rc == HSF_OK) rc = nalloc(n, n->allocs, (void **)&n->m, sizeof(float) * off);
    if (rc == HSF_OK) rc = nalloc(n, n->allocs, (void **)&n->v, sizeof(float) * off);
    if (rc == HSF_OK) rc = nalloc(n, n->allocs, (void **)&n->norm, sizeof(float) * 2 * in_ch);
    for (int l = 0; l < kLayers && rc == HSF_OK; ++l) {
        Layer &Ly = n->layer[l];
        rc = nalloc(n, n->allocs, (void **)&Ly.Wm, sizeof(__bf16) * (size_t)Ly.cop * Ly.kp);
        if (rc == HSF_OK) rc = nalloc(n, n->allocs, (void **)&Ly.Wt, sizeof(__bf16) * (size_t)Ly.cop_t * Ly.kp_t);
        if (rc == HSF_OK) rc = nalloc(n, n->allocs, (void **)&Ly.dWm, sizeof(float) * (size_t)Ly.cop * Ly.kp);
    }
    if (rc != HSF_OK) {
        hsf_net_destroy(n);
        return rc;
    }
    std::vector<float> p(off, 0.0f);
    for (int l = 0; l < kLayers; ++l) {
        const Layer &Ly = n->layer[l];
        double a = sqrt(3.0 / (27.0 * Ly.ci));
        if (l == kLayers - 1) a *= 0.25;
        for (long long i = 0; i < (long long)Ly.co * Ly.ci * 27; ++i)
            p[Ly.w_off + i] = (float)(a * (2.0 * unit_hash(seed, Ly.w_off + i) - 1.0));
    }
    std::vector<float> nrm(2 * in_ch, 0.0f);
    for (int c = 0; c < in_ch; ++c) nrm[in_ch + c] = 1.0f;   // identity normalisation
    hipError_t e = hipMemcpy(n->params, p.data(), sizeof(float) * off, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->norm, nrm.data(), sizeof(float) * 2 * in_ch, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->m, 0, sizeof(float) * off);
    if (e == hipSuccess) e = hipMemset(n->v, 0, sizeof(float) * off);
    if (e == hipSuccess) e = hipMemset(n->grad, 0, sizeof(float) * off);
    if (e != hipSuccess) {
        hsf_net_destroy(n);
        return HSF_EHIP;
    }
    *out = n;
    return HSF_OK;
}

void hsf_net_destroy(hsf_net *n)
{
    if (!n) return;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    else (void)hipDeviceSynchronize();
    free_acts(n);
    for (void *p : n->allocs) (void)hipFree(p);
    delete n;
}

const char *hsf_net_last_error(const hsf_net *n) { return n ? n->err.c_str() : "null network"; }

int hsf_net_set_stream(hsf_net *n, void *stream)
{
    if (!n) return HSF_EINVAL;
    n->stream = (hipStream_t)stream;
    return HSF_OK;
}

long long hsf_net_num_params(const hsf_net *n) { return n ? n->n_params : -1; }

int hsf_net_set_params(hsf_net *n, const float *p, int where)
{
    if (!n) return HSF_EINVAL;
    int rc = copy_f32(n, n->params, p, n->n_params, where, hipMemcpyHostToDevice);
    if (rc) return rc;
    n->adam_t = 0;
    NCHK(n, hipMemsetAsync(n->m, 0, sizeof(float) * n->n_params, n->stream));
    NCHK(n, hipMemsetAsync(n->v, 0, sizeof(float) * n->n_params, n->stream));
    return stage_weights(n);
}

int hsf_net_set_input_norm(hsf_net *n, const float *shift, const float *scale)
{
    if (!n || !shift || !scale) return HSF_EINVAL;
    std::vector<float> nrm(2 * n->in_ch);
    for (int c = 0; c < n->in_ch; ++c) {
        nrm[c] = shift[c];
        nrm[n->in_ch + c] = scale[c];
    }
    NCHK(n, hipMemcpyAsync(n->norm, nrm.data(), sizeof(float) * nrm.size(), hipMemcpyHostToDevice, n->stream));
    NCHK(n, hipStreamSynchronize(n->stream));
    return HSF_OK;
}

int hsf_net_get_params(hsf_net *n, float *p, int where)
{
    if (!n) return HSF_EINVAL;
    return copy_f32(n, p, n->params, n->n_params, where, hipMemcpyDeviceToHost);
}

int hsf_net_forward(hsf_net *n, const float *in, float *out, int batch, int L, int where)
{
    if (!n) return HSF_EINVAL;
    int rc = check_box(n, batch, L);
    if (rc) return rc;
    if ((rc = ensure_acts(n, batch, L, false))) return rc;
    if (!n->weights_staged && (rc = stage_weights(n))) return rc;
    if ((rc = copy_f32(n, n->x0.p, in, (size_t)batch * n->in_ch * vol(L, 0), where, hipMemcpyHostToDevice)))
        return rc;
    forward(n);
    NCHK(n, hipGetLastError());
    return copy_f32(n, out, n->y[14].p, (size_t)batch * n->out_ch * vol(L, 0), where, hipMemcpyDeviceToHost);
}

int hsf_net_loss_grad(hsf_net *n, const float *in, const float *target, int batch, int L, double *loss, float *grad,
                      int where)
{
    if (!n) return HSF_EINVAL;
    int rc = check_box(n, batch, L);
    if (rc) return rc;
    if ((rc = ensure_acts(n, batch, L, true))) return rc;
    const size_t nin = (size_t)batch * n->in_ch * vol(L, 0), nout = (size_t)batch * n->out_ch * vol(L, 0);
    if ((rc = copy_f32(n, n->x0.p, in, nin, where, hipMemcpyHostToDevice))) return rc;
    if ((rc = copy_f32(n, n->target, target, nout, where, hipMemcpyHostToDevice))) return rc;
    if ((rc = loss_and_grad(n, loss))) return rc;
    if (grad) return copy_f32(n, grad, n->grad, n->n_params, where, hipMemcpyDeviceToHost);
    return HSF_OK;
}

int hsf_net_train_step(hsf_net *n, const float *in, const float *target, int batch, int L, float lr, double *loss,
                       int where)
{
    int rc = hsf_net_loss_grad(n, in, target, batch, L, loss, nullptr, where);
    if (rc) return rc;
    n->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)n->adam_t), c2 = 1.0f - powf(b2, (float)n->adam_t);
    net_adam(n->stream, n->params, n->grad, n->m, n->v, n->n_params, lr, b1, b2, 1e-8f, c1, c2);
    return stage_weights(n);
}

}  // extern "C"

// ---- use by the inversion (called from api.hip) ------------------------------------

namespace hsf {

// Prediction for one replica: x is the prepared FP32 input [in_ch][V] (device), pred
// receives [out_ch][V] FP32 (device).  Returns an HSF code.
int net_predict(hsf_net *n, hipStream_t s, const float *x, int in_ch, int L, float *pred)
{
    if (!n || in_ch != n->in_ch) return HSF_EINVAL;
    int rc = check_box(n, 1, L);
    if (rc) return rc;
    hipStream_t saved = n->stream;
    n->stream = s;
    if ((rc = ensure_acts(n, 1, L, false)) || (!n->weights_staged && (rc = stage_weights(n)))) {
        n->stream = saved;
        return rc;
    }
    hipError_t e = hipMemcpyAsync(n->x0.p, x, sizeof(float) * in_ch * vol(L, 0), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) {
        forward(n);
        e = hipMemcpyAsync(pred, n->y[14].p, sizeof(float) * n->out_ch * vol(L, 0), hipMemcpyDeviceToDevice, s);
    }
    n->stream = saved;
    return e == hipSuccess ? HSF_OK : HSF_EHIP;
}

int net_channels(const hsf_net *n, int *in_ch, int *out_ch)
{
    if (!n) return HSF_EINVAL;
    *in_ch = n->in_ch;
    *out_ch = n->out_ch;
    return HSF_OK;
}

}  // namespace hsf
