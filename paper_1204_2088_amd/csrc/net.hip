// net.hip -- the warm-start network (a build addition to the method): a U-Net of
// D = 1..4 levels on the periodic lattice, trained on pairs produced by the
// inversion itself.  Forward and backward passes run in the kernels of
// net_kernels.hip (convolutions on the BF16 matrix cores, FP32 accumulation);
// master weights and Adam moments are FP32.
//
// Topology (widths w1..wD, SiLU after every convolution except the last):
//   e1 = c(c(x, in->w1), w1->w1)                              level 0 (box L)
//   el = c(c(pool e(l-1), w(l-1)->wl), wl->wl)                level l-1 (box L / 2^(l-1))
//   dD = eD;  dl = c(c(up d(l+1), w(l+1)->wl) + el, wl->wl)   for l = D-1 .. 1
//   out = conv(d1, w1->out)                                   level 0, no activation
// c(.) = SiLU(3x3x3 periodic convolution + bias); pool = 2x2x2 average; up = nearest.
// Pooled, upsampled and skip-summed inputs are composed while a convolution stages
// its tile (ConvIn), never stored.  4 D - 1 convolutions; parameter vector: for each
// in the order above (encoder, decoder from the coarsest level, output), W[co][ci][27]
// then b[co].
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "hsf.h"
#include "net_internal.h"

using namespace hsf;

namespace {

constexpr int kMaxLevels = 4;
// auxiliary device scratch of a network: 4096 partial sums, then results
constexpr int kAuxParts = 4096, kAuxDoubles = kAuxParts + 8 + 2 * 64 + 64;
constexpr int kLayers = 4 * kMaxLevels - 1;   // the most convolutions a network has

int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct Layer {
    int ci, co, act, level;          // level 0..D-1 (box L >> level)
    int cip, kp, cop;                // forward matrix-core layout
    int cip_t, kp_t, cop_t;          // transposed-flipped layout (data gradient)
    long long w_off, b_off;          // offsets in the parameter vector
    // input composition: mode (CONV_IN_*) and the activations it reads (-1: network input)
    int in_mode, src1, src2;
    // inference keeps the activation packed (BF16 [batch][site][cip of its readers]):
    // every layer that reads it reads it plainly
    int pack = 0;
    __bf16 *Wm = nullptr, *Wt = nullptr;
    float *dWm = nullptr;            // weight gradient, matrix-core layout
};

struct Tensor {
    float *p = nullptr;
    __bf16 *pk = nullptr;   // packed BF16 copy used by inference (activations with Layer::pack)
    int c = 0, level = 0;
};

}  // namespace

struct hsf_net {
    int in_ch = 0, out_ch = 0, w[kMaxLevels] = {0, 0, 0, 0};
    int depth = 0, n_layers = 0;
    Layer layer[kLayers];
    long long n_params = 0;
    float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    float *norm = nullptr;           // device: input shift[in_ch], scale[in_ch], output zero[out_ch], scale[out_ch]
    int out_scaled = 0;              // an output scale other than 1 is set
    long long adam_t = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<void *> allocs;      // parameter-sized and weight buffers
    // activation buffers for the current (batch, box)
    int cur_B = 0, cur_L = 0;
    std::vector<void *> act_allocs;
    Tensor x0, y[kLayers], a[kLayers];
    Tensor dy[kLayers], da[kLayers], dout;
    float *din = nullptr;            // gradient of one convolution's (composed) input
    float *target = nullptr, *wpart = nullptr;
    double *bpart = nullptr;         // per-channel partial sums of the bias gradient
    double *loss_part = nullptr;
    double *aux = nullptr;           // sample assembly and channel moments: partials, rms, results
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
    n->x0 = n->dout = Tensor();
    for (int l = 0; l < kLayers; ++l) n->y[l] = n->a[l] = n->dy[l] = n->da[l] = Tensor();
    n->din = n->target = n->wpart = nullptr;
    n->bpart = nullptr;
    n->loss_part = nullptr;
}

// Elements of a layer's (composed) input for the current batch.
long long input_numel(const hsf_net *n, const Layer &Ly)
{
    return (long long)n->cur_B * Ly.ci * vol(n->cur_L, Ly.level);
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
    T(n->x0, n->in_ch, 0);
    for (int l = 0; l < n->n_layers; ++l) {
        const Layer &Ly = n->layer[l];
        // pre-activations are kept for the backward pass and for the output layer;
        // FP32 activations for the backward pass and for readers that compose them
        if (grads || !Ly.act) T(n->y[l], Ly.co, Ly.level);
        if (Ly.act && (grads || !Ly.pack)) T(n->a[l], Ly.co, Ly.level);
        if (Ly.pack && rc == HSF_OK) {   // always there, so inference after training finds it
            n->a[l].c = Ly.co;
            n->a[l].level = Ly.level;
            rc = nalloc(n, n->act_allocs, (void **)&n->a[l].pk,
                        sizeof(__bf16) * (size_t)B * round_up(Ly.co, 8) * vol(L, Ly.level));
        }
    }
    if (grads) {
        size_t din = 0, wp = 0;
        for (int l = 0; l < n->n_layers; ++l) {
            const Layer &Ly = n->layer[l];
            T(n->dy[l], Ly.co, Ly.level);
            if (Ly.act) T(n->da[l], Ly.co, Ly.level);
            din = std::max(din, (size_t)((long long)B * Ly.ci * vol(L, Ly.level)));
            wp = std::max(wp, (size_t)net_wgrad_slices(B, L >> Ly.level, Ly.cop, Ly.kp) * Ly.cop * Ly.kp);
        }
        T(n->dout, n->out_ch, 0);
        if (rc == HSF_OK) rc = nalloc(n, n->act_allocs, (void **)&n->din, sizeof(float) * din);
        if (rc == HSF_OK)
            rc = nalloc(n, n->act_allocs, (void **)&n->target, sizeof(float) * (size_t)B * n->out_ch * vol(L, 0));
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
    for (int l = 0; l < n->n_layers; ++l) {
        const Layer &Ly = n->layer[l];
        net_stage_weights(n->stream, n->params + Ly.w_off, Ly.co, Ly.ci, Ly.cip, Ly.kp, Ly.cop, Ly.Wm, Ly.cip_t,
                          Ly.kp_t, Ly.cop_t, Ly.Wt);
    }
    NCHK(n, hipGetLastError());
    n->weights_staged = 1;
    return HSF_OK;
}

const float *src_ptr(const hsf_net *n, int src) { return src < 0 ? n->x0.p : n->a[src].p; }

ConvIn conv_input(const hsf_net *n, const Layer &Ly)
{
    ConvIn in;
    in.x1 = src_ptr(n, Ly.src1);
    in.x2 = Ly.in_mode == CONV_IN_ADD ? src_ptr(n, Ly.src2) : nullptr;
    in.mode = Ly.in_mode;
    return in;
}

// Forward of layer l.  Training keeps the FP32 pre-activation and activation for the
// backward pass, reading the normalised input x0.  Inference writes the activation
// alone (packed when every reader reads it plainly), reads the network input x (with
// the input normalisation applied while staging) and writes the output layer, with
// the output scale applied, to y.
void conv(hsf_net *n, int l, const float *x, float *y)
{
    const Layer &Ly = n->layer[l];
    ConvIn in = conv_input(n, Ly);
    ConvOut out;
    if (n->training) {
        out.Y = n->y[l].p;
        out.A = Ly.act ? n->a[l].p : nullptr;
    } else {
        if (Ly.src1 < 0) {
            in.x1 = x;
            in.shift = n->norm;
            in.scale = n->norm + n->in_ch;
        } else if (n->layer[Ly.src1].pack) {
            in.mode = CONV_IN_PACKED;
            in.x1 = nullptr;
            in.xp = n->a[Ly.src1].pk;
        }
        if (Ly.pack) {
            out.Ap = n->a[l].pk;
        } else if (Ly.act) {
            out.A = n->a[l].p;
        } else {
            out.Y = y;
            if (n->out_scaled) {
                out.shift = n->norm + 2 * n->in_ch;
                out.scale = out.shift + n->out_ch;
            }
        }
    }
    net_conv_fwd(n->stream, in, n->cur_B, Ly.ci, Ly.cip, Ly.Wm, Ly.kp, Ly.co, Ly.cop, n->params + Ly.b_off, out,
                 n->cur_L >> Ly.level);
}

long long numel(const hsf_net *n, const Tensor &t) { return (long long)n->cur_B * t.c * vol(n->cur_L, t.level); }

const Tensor &output(const hsf_net *n) { return n->y[n->n_layers - 1]; }

// Training forward pass: normalises x0 in place (the weight gradient of the first
// layer reads it) and keeps every layer's FP32 tensors.  The output scale is 1 here.
void forward_train(hsf_net *n)
{
    net_affine(n->stream, n->x0.p, n->in_ch, vol(n->cur_L, 0), numel(n, n->x0), n->norm, n->norm + n->in_ch);
    for (int l = 0; l < n->n_layers; ++l) conv(n, l, nullptr, nullptr);
}

// Inference: network input x ([B][in_ch][V] FP32, not modified) to output y
// ([B][out_ch][V] FP32).  x is read with 16-byte vector loads where the box allows, so
// an input that is not 16-byte aligned is copied to x0 first.
int forward_infer(hsf_net *n, const float *x, float *y)
{
    if (reinterpret_cast<uintptr_t>(x) % 16 != 0) {
        NCHK(n, hipMemcpyAsync(n->x0.p, x, sizeof(float) * numel(n, n->x0), hipMemcpyDeviceToDevice, n->stream));
        x = n->x0.p;
    }
    for (int l = 0; l < n->n_layers; ++l) conv(n, l, x, y);
    NCHK(n, hipGetLastError());
    return HSF_OK;
}

// Backward pass from dout (gradient of the loss with respect to the output).  Layers
// are visited from the last; every consumer of an activation comes after it, so
// da[j] is complete when layer j is reached.  dgrad writes the gradient of a layer's
// composed input into din, which is then distributed to the activations it read.
void backward(hsf_net *n)
{
    hipStream_t s = n->stream;
    const int B = n->cur_B, L = n->cur_L;
    bool have[kLayers] = {false};
    for (int l = n->n_layers - 1; l >= 0; --l) {
        const Layer &Ly = n->layer[l];
        const int Ll = L >> Ly.level;
        const long long V = vol(L, Ly.level);
        if (Ly.act) {
            net_silu_bwd(s, n->da[l].p, n->y[l].p, n->dy[l].p, numel(n, n->dy[l]));
        } else {
            (void)hipMemcpyAsync(n->dy[l].p, n->dout.p, sizeof(float) * numel(n, n->dout), hipMemcpyDeviceToDevice,
                                 s);
        }
        net_conv_wgrad(s, conv_input(n, Ly), B, Ly.ci, Ly.cip, n->dy[l].p, Ly.co, Ly.cop, Ly.kp, Ll, n->wpart,
                       Ly.dWm);
        net_unstage_grad(s, Ly.dWm, Ly.co, Ly.ci, Ly.cip, Ly.kp, n->grad + Ly.w_off);
        net_channel_sum(s, n->dy[l].p, B, Ly.co, V, n->bpart, n->grad + Ly.b_off);
        if (Ly.src1 < 0) continue;   // the network input needs no gradient
        ConvIn g;
        g.x1 = n->dy[l].p;
        ConvOut gout;
        gout.Y = n->din;
        net_conv_fwd(s, g, B, Ly.co, Ly.cip_t, Ly.Wt, Ly.kp_t, Ly.ci, Ly.cop_t, nullptr, gout, Ll);
        const long long nin = input_numel(n, Ly);
        auto give = [&](int j) {   // da[j] (+)= din through the input's composition
            float *dst = n->da[j].p;
            const int add = have[j] ? 1 : 0;
            if (Ly.in_mode == CONV_IN_UP)
                net_up_bwd(s, n->din, dst, Ll, numel(n, n->da[j]), add);
            else if (Ly.in_mode == CONV_IN_POOL)
                net_pool_bwd(s, n->din, dst, L >> n->layer[j].level, numel(n, n->da[j]), add);
            else
                net_accum(s, dst, n->din, nin, add);
            have[j] = true;
        };
        give(Ly.src1);
        if (Ly.in_mode == CONV_IN_ADD) give(Ly.src2);
    }
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
    const int q = 1 << (n->depth - 1);
    if (B < 1 || L < q || (L % q) != 0)
        return nfail(n, HSF_EINVAL, "batch %d, box %d: need L a multiple of %d", B, L, q);
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
    if (n->out_scaled) return nfail(n, HSF_EINVAL, "training needs the output scale reset to 1");
    n->training = 1;
    forward_train(n);
    n->training = 0;
    const long long cnt = numel(n, n->dout);
    const int blocks = net_mse(n->stream, output(n).p, n->target, n->dout.p, cnt, 1.0f / (float)cnt, n->loss_part);
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
    int D = 0;
    while (D < kMaxLevels && widths[D] > 0) ++D;
    if (D == 0) return HSF_EINVAL;
    for (int i = 0; i < kMaxLevels; ++i)
        if (widths[i] > kNetMaxWidth || widths[i] < 0 || (i >= D && widths[i] != 0)) return HSF_EINVAL;
    hsf_net *n = new hsf_net();
    n->in_ch = in_ch;
    n->out_ch = out_ch;
    n->depth = D;
    for (int i = 0; i < kMaxLevels; ++i) n->w[i] = widths[i];
    const int *w = widths;
    int nl = 0;
    auto add = [&](int ci, int co, int act, int level, int mode, int src1, int src2) {
        Layer &Ly = n->layer[nl++];
        Ly.ci = ci;
        Ly.co = co;
        Ly.act = act;
        Ly.level = level;
        Ly.in_mode = mode;
        Ly.src1 = src1;
        Ly.src2 = src2;
    };
    for (int lev = 0; lev < D; ++lev) {   // encoder: e(lev+1) = activation of layer 2 lev + 1
        if (lev == 0) add(in_ch, w[0], 1, 0, CONV_IN_PLAIN, -1, -1);
        else add(w[lev - 1], w[lev], 1, lev, CONV_IN_POOL, 2 * lev - 1, -1);
        add(w[lev], w[lev], 1, lev, CONV_IN_PLAIN, nl - 1, -1);
    }
    int prev = 2 * D - 1;                 // d(D) = e(D)
    for (int lev = D - 2; lev >= 0; --lev) {
        add(w[lev + 1], w[lev], 1, lev, CONV_IN_UP, prev, -1);
        add(w[lev], w[lev], 1, lev, CONV_IN_ADD, nl - 1, 2 * lev + 1);
        prev = nl - 1;
    }
    add(w[0], out_ch, 0, 0, CONV_IN_PLAIN, prev, -1);
    n->n_layers = nl;
    for (int l = 0; l < nl; ++l) {   // activations whose readers all read them plainly
        Layer &Ly = n->layer[l];
        int readers = 0, plain = 0;
        for (int j = 0; j < nl; ++j) {
            const Layer &R = n->layer[j];
            const bool reads = R.src1 == l || (R.in_mode == CONV_IN_ADD && R.src2 == l);
            readers += reads;
            plain += reads && R.in_mode == CONV_IN_PLAIN;
        }
        Ly.pack = Ly.act && readers > 0 && plain == readers;
    }
    long long off = 0;
    for (int l = 0; l < nl; ++l) {
        Layer &Ly = n->layer[l];
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
    if (rc == HSF_OK) rc = nalloc(n, n->allocs, (void **)&n->norm, sizeof(float) * 2 * (in_ch + out_ch));
    if (rc == HSF_OK) rc = nalloc(n, n->allocs, (void **)&n->aux, sizeof(double) * kAuxDoubles);
    for (int l = 0; l < n->n_layers && rc == HSF_OK; ++l) {
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
    for (int l = 0; l < n->n_layers; ++l) {
        const Layer &Ly = n->layer[l];
        double a = sqrt(3.0 / (27.0 * Ly.ci));
        if (l == n->n_layers - 1) a *= 0.25;
        for (long long i = 0; i < (long long)Ly.co * Ly.ci * 27; ++i)
            p[Ly.w_off + i] = (float)(a * (2.0 * unit_hash(seed, Ly.w_off + i) - 1.0));
    }
    std::vector<float> nrm(2 * (in_ch + out_ch), 0.0f);   // identity normalisation and scale
    for (int c = 0; c < in_ch; ++c) nrm[in_ch + c] = 1.0f;
    for (int c = 0; c < out_ch; ++c) nrm[2 * in_ch + out_ch + c] = 1.0f;
    hipError_t e = hipMemcpy(n->params, p.data(), sizeof(float) * off, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->norm, nrm.data(), sizeof(float) * nrm.size(), hipMemcpyHostToDevice);
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

int hsf_net_set_output_scale(hsf_net *n, const float *scale)
{
    if (!n || !scale) return HSF_EINVAL;
    std::vector<float> v(2 * n->out_ch, 0.0f);
    int scaled = 0;
    for (int c = 0; c < n->out_ch; ++c) {
        v[n->out_ch + c] = scale[c];
        scaled |= scale[c] != 1.0f;
    }
    NCHK(n, hipMemcpyAsync(n->norm + 2 * n->in_ch, v.data(), sizeof(float) * v.size(), hipMemcpyHostToDevice,
                           n->stream));
    NCHK(n, hipStreamSynchronize(n->stream));
    n->out_scaled = scaled;
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
    if (!in || !out) return nfail(n, HSF_EINVAL, "null pointer");
    if (where == HSF_DEVICE) return forward_infer(n, in, out);   // straight from and into the caller's buffers
    if ((rc = copy_f32(n, n->x0.p, in, (size_t)batch * n->in_ch * vol(L, 0), where, hipMemcpyHostToDevice)))
        return rc;
    if ((rc = forward_infer(n, n->x0.p, output(n).p))) return rc;
    return copy_f32(n, out, output(n).p, (size_t)batch * n->out_ch * vol(L, 0), where, hipMemcpyDeviceToHost);
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

int hsf_net_make_sample(hsf_net *n, const double *phi, const double *phi_n, const double *phi_p, const double *w,
                        const double *w_n, const double *w_p, int nsp, long long V, int mode, float *x, float *y)
{
    if (!n) return HSF_EINVAL;
    if (!phi || !w || !x || !y || (mode >= 1 && (!phi_n || !w_n)) || (mode == 2 && (!phi_p || !w_p)) || mode < 0 ||
        mode > 2 || (nsp != 2 && nsp != 3) || V < 1)
        return nfail(n, HSF_EINVAL, "bad sample arguments");
    if (mode == 0) {   // the direct map: only the step's own state is read
        phi_n = phi_p = phi;
        w_n = w_p = w;
    }
    net_sample(n->stream, phi, phi_n, mode == 2 ? phi_p : phi_n, w, w_n, mode == 2 ? w_p : w_n, nsp, V, mode, n->aux,
               kAuxParts, n->aux + kAuxParts, x, y);
    NCHK(n, hipGetLastError());
    return HSF_OK;
}

int hsf_net_affine(hsf_net *n, float *x, int batch, int channels, long long V, const float *shift,
                   const float *scale)
{
    if (!n) return HSF_EINVAL;
    if (!x || !shift || !scale || batch < 1 || channels < 1 || channels > 64 || V < 1)
        return nfail(n, HSF_EINVAL, "bad affine arguments");
    std::vector<float> h(2 * channels);
    for (int c = 0; c < channels; ++c) {
        h[c] = shift[c];
        h[channels + c] = scale[c];
    }
    float *d = reinterpret_cast<float *>(n->aux + kAuxParts + 8 + 2 * 64);   // 2 x 64 floats fit in 64 doubles
    NCHK(n, hipMemcpyAsync(d, h.data(), sizeof(float) * 2 * channels, hipMemcpyHostToDevice, n->stream));
    net_affine(n->stream, x, channels, V, (long long)batch * channels * V, d, d + channels);
    NCHK(n, hipGetLastError());
    NCHK(n, hipStreamSynchronize(n->stream));   // the host staging array goes out of scope
    return HSF_OK;
}

int hsf_net_channel_moments(hsf_net *n, const float *x, int batch, int channels, long long V, double *mean,
                            double *rms)
{
    if (!n) return HSF_EINVAL;
    if (!x || !mean || !rms || batch < 1 || channels < 1 || channels > 64 || V < 1)
        return nfail(n, HSF_EINVAL, "bad moment arguments");
    const int nblk = std::max(1, kAuxParts / (2 * channels));
    double *out = n->aux + kAuxParts + 8;
    net_channel_moments(n->stream, x, batch, channels, V, n->aux, nblk, out);
    NCHK(n, hipGetLastError());
    std::vector<double> h(2 * channels);
    NCHK(n, hipMemcpyAsync(h.data(), out, sizeof(double) * 2 * channels, hipMemcpyDeviceToHost, n->stream));
    NCHK(n, hipStreamSynchronize(n->stream));
    for (int c = 0; c < channels; ++c) {
        mean[c] = h[2 * c];
        rms[c] = h[2 * c + 1];
    }
    return HSF_OK;
}

}  // extern "C"

// ---- use by the inversion (called from api.hip) ------------------------------------

namespace hsf {

// Prediction for B samples (replicas) on an L^3 box: x is the prepared FP32 input
// [B][in_ch][V] (device), pred receives [B][out_ch][V] FP32 (device).  Returns an HSF
// code.
int net_predict(hsf_net *n, hipStream_t s, const float *x, int in_ch, int B, int L, float *pred)
{
    if (!n || in_ch != n->in_ch) return HSF_EINVAL;
    int rc = check_box(n, B, L);
    if (rc) return rc;
    hipStream_t saved = n->stream;
    n->stream = s;
    if ((rc = ensure_acts(n, B, L, false)) || (!n->weights_staged && (rc = stage_weights(n)))) {
        n->stream = saved;
        return rc;
    }
    rc = forward_infer(n, x, pred);
    n->stream = saved;
    return rc;
}

int net_channels(const hsf_net *n, int *in_ch, int *out_ch, int *box_multiple)
{
    if (!n) return HSF_EINVAL;
    *in_ch = n->in_ch;
    *out_ch = n->out_ch;
    *box_multiple = 1 << (n->depth - 1);
    return HSF_OK;
}

}  // namespace hsf
