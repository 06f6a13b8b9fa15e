// net_kernels.hip -- kernels of the warm-start network: periodic 3x3x3
// convolutions as implicit GEMMs on the BF16 matrix cores (FP32 accumulation),
// the weight gradient as a second MFMA GEMM over sites, and the element-wise
// parts (activation, pooling, upsampling, skip sums, loss, Adam).
//
// Tensors are FP32 [batch][channel][site] with site = x + L (y + L z) on a
// periodic L^3 box.  A convolution layer's weights W[co][ci][k] (k = 9 (dz+1) +
// 3 (dy+1) + (dx+1)) are staged for the matrix cores as BF16 rows
// Wm[co][kk], kk = k * cip + ci (cip = ci rounded up to 8), zero beyond 27 cip
// and up to kp = a multiple of 32, and co padded to a multiple of 16.
//
// v_mfma_f32_16x16x32_bf16 lane layout (wave of 64): A (16 x 32): lane l holds
// row l % 16, k = 8 (l / 16) + j; B (32 x 16): column l % 16, same k; C (16 x 16):
// column l % 16, rows 4 (l / 16) + i.
#include <hip/hip_ext.h>
#include <math.h>

#include "net_internal.h"

namespace hsf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wrapL(int v, int L)
{
    v %= L;
    return v < 0 ? v + L : v;
}

__device__ __forceinline__ float silu(float y) { return y / (1.0f + __expf(-y)); }
__device__ __forceinline__ float silu_grad(float y)
{
    const float s = 1.0f / (1.0f + __expf(-y));
    return s * (1.0f + y * (1.0f - s));
}

// ---------------------------------------------------------------- forward convolution
// Y[b][co][x] = bias[co] + sum_{ci,k} W[co][ci][k] X[b][ci][x + off_k]; optional
// A = silu(Y).  Block: a TX x TY x TZ tile of one sample (128 sites, 8 MFMA column
// tiles, two per wave); the input tile with a one-site halo is staged in LDS as BF16
// [halo site][cip].
constexpr int TX = 8, TY = 4, TZ = 4, TS = TX * TY * TZ;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HS = HX * HY * HZ;

__global__ __launch_bounds__(256) void k_conv_fwd(const float *__restrict__ X, int ci, int cip,
                                                   const __bf16 *__restrict__ Wm, int kp, int co, int cop,
                                                   const float *__restrict__ bias, float *__restrict__ Y,
                                                   float *__restrict__ A, int L, int tiles_x, int tiles_y,
                                                   int tiles_per_sample)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16 *xs = reinterpret_cast<__bf16 *>(smem);   // [HS][cip]
    const int b = blockIdx.x / tiles_per_sample;
    int t = blockIdx.x % tiles_per_sample;
    const int x0 = (t % tiles_x) * TX;
    t /= tiles_x;
    const int y0 = (t % tiles_y) * TY;
    const int z0 = (t / tiles_y) * TZ;
    const long long V = (long long)L * L * L;
    const float *Xb = X + (long long)b * ci * V;
    // stage the halo tile
    for (int e = threadIdx.x; e < HS * cip; e += 256) {
        const int h = e % HS, c = e / HS;
        const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
        float v = 0.0f;
        if (c < ci) {
            const int gx = wrapL(x0 + hx - 1, L), gy = wrapL(y0 + hy - 1, L), gz = wrapL(z0 + hz - 1, L);
            v = Xb[(long long)c * V + gx + (long long)L * (gy + (long long)L * gz)];
        }
        xs[h * cip + c] = (__bf16)v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane >> 4, col = lane & 15;
    const int nmt = cop / 16;
    floatx4 acc[2][4];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[q][m] = floatx4{0.f, 0.f, 0.f, 0.f};
    // this lane's two sites (column of the B operand), as halo-tile positions
    int hbase[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int n = (wave * 2 + q) * 16 + col;
        const int tx = n % TX, ty = (n / TX) % TY, tz = n / (TX * TY);
        hbase[q] = (tz + 1) * HX * HY + (ty + 1) * HX + (tx + 1);
    }
    for (int kc = 0; kc < kp; kc += 32) {
        const int kk = kc + 8 * grp;
        int k = kk / cip;
        const int c0 = kk - k * cip;
        if (k > 26) k = 13;   // padding rows of K: zero weights, any finite input
        const int off = ((k / 9) - 1) * HX * HY + (((k / 3) % 3) - 1) * HX + ((k % 3) - 1);
        bf16x8 bv[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) bv[q] = *reinterpret_cast<const bf16x8 *>(xs + (hbase[q] + off) * cip + c0);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (m >= nmt) break;
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(Wm + (long long)(m * 16 + col) * kp + kk);
#pragma unroll
            for (int q = 0; q < 2; ++q)
                acc[q][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[q], acc[q][m], 0, 0, 0);
        }
    }
    // epilogue: lane holds rows 4 grp + i of each M tile, column = its site
    float *Yb = Y + (long long)b * co * V;
    float *Ab = A ? A + (long long)b * co * V : nullptr;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int n = (wave * 2 + q) * 16 + col;
        const int tx = n % TX, ty = (n / TX) % TY, tz = n / (TX * TY);
        const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
        if (gx >= L || gy >= L || gz >= L) continue;
        const long long site = gx + (long long)L * (gy + (long long)L * gz);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (m >= nmt) break;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = m * 16 + 4 * grp + i;
                if (o >= co) continue;
                const float y = acc[q][m][i] + (bias ? bias[o] : 0.0f);
                Yb[(long long)o * V + site] = y;
                if (Ab) Ab[(long long)o * V + site] = silu(y);
            }
        }
    }
}

// ---------------------------------------------------------------- weight gradient
// dW[co][k cip + ci] = sum_b sum_x dY[b][co][x] X[b][ci][x + off_k], as the GEMM
// C (cop x kp) = A (cop x sites) B (sites x kp).  Block (g, sp): the 16 C tiles of
// group g (4 per wave, accumulated in registers) over the site tiles sp, sp + nsp, ...
// (K chunks of 32 sites = 4 x-rows of 8).  Partial C per site slice goes to `part`
// [sp][cop][kp] and is summed in a fixed order by k_sum_blocks.
constexpr int WG_TILES_PER_WAVE = 4;

__global__ __launch_bounds__(256) void k_conv_wgrad(const float *__restrict__ X, int ci, int cip,
                                                     const float *__restrict__ dY, int co, int cop, int kp,
                                                     int L, int tiles_x, int tiles_y, int tiles_per_sample,
                                                     int n_tiles, int n_groups, int n_slices,
                                                     float *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16 *xs = reinterpret_cast<__bf16 *>(smem);      // [cip][HS]   (site fastest)
    __bf16 *ys = xs + (size_t)cip * HS;                 // [cop][TS]
    const int g = blockIdx.x % n_groups, sp = blockIdx.x / n_groups;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane >> 4, col = lane & 15;
    const int nnt = kp / 16, ntiles = (cop / 16) * nnt;
    const long long V = (long long)L * L * L;
    floatx4 acc[WG_TILES_PER_WAVE];
#pragma unroll
    for (int j = 0; j < WG_TILES_PER_WAVE; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int tile = sp; tile < n_tiles; tile += n_slices) {
        const int b = tile / tiles_per_sample;
        int t = tile % tiles_per_sample;
        const int x0 = (t % tiles_x) * TX;
        t /= tiles_x;
        const int y0 = (t % tiles_y) * TY;
        const int z0 = (t / tiles_y) * TZ;
        __syncthreads();
        for (int e = threadIdx.x; e < HS * cip; e += 256) {
            const int h = e % HS, c = e / HS;
            const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
            float v = 0.0f;
            if (c < ci) {
                const int gx = wrapL(x0 + hx - 1, L), gy = wrapL(y0 + hy - 1, L), gz = wrapL(z0 + hz - 1, L);
                v = X[((long long)b * ci + c) * V + gx + (long long)L * (gy + (long long)L * gz)];
            }
            xs[c * HS + h] = (__bf16)v;
        }
        for (int e = threadIdx.x; e < TS * cop; e += 256) {
            const int n = e % TS, o = e / TS;
            const int tx = n % TX, ty = (n / TX) % TY, tz = n / (TX * TY);
            const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
            float v = 0.0f;
            if (o < co && gx < L && gy < L && gz < L)   // sites outside the box contribute nothing
                v = dY[((long long)b * co + o) * V + gx + (long long)L * (gy + (long long)L * gz)];
            ys[o * TS + n] = (__bf16)v;
        }
        __syncthreads();
        for (int kc = 0; kc < TS; kc += 32) {
            // 8 consecutive sites of this lane group: one x-row of the tile
            const int s0 = kc + 8 * grp;
            const int ty = (s0 / TX) % TY, tz = s0 / (TX * TY);
#pragma unroll
            for (int j = 0; j < WG_TILES_PER_WAVE; ++j) {
                const int tix = g * 16 + wave * WG_TILES_PER_WAVE + j;
                if (tix < ntiles) {
                    const int m = tix / nnt, nt = tix % nnt;
                    const bf16x8 av = *reinterpret_cast<const bf16x8 *>(ys + (m * 16 + col) * TS + s0);
                    const int kk = nt * 16 + col;
                    int k = kk / cip;
                    const int c = kk - k * cip;
                    bf16x8 bv;
                    if (k > 26) {
#pragma unroll
                        for (int q = 0; q < 8; ++q) bv[q] = (__bf16)0.0f;
                    } else {
                        const int dx = (k % 3) - 1, dy = ((k / 3) % 3) - 1, dz = (k / 9) - 1;
                        const __bf16 *row = xs + c * HS + (tz + 1 + dz) * HX * HY + (ty + 1 + dy) * HX + 1 + dx;
#pragma unroll
                        for (int q = 0; q < 8; ++q) bv[q] = row[q];
                    }
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[j], 0, 0, 0);
                }
            }
        }
    }
    float *P = part + (long long)sp * cop * kp;
#pragma unroll
    for (int j = 0; j < WG_TILES_PER_WAVE; ++j) {
        const int tix = g * 16 + wave * WG_TILES_PER_WAVE + j;
        if (tix < ntiles) {
            const int m = tix / nnt, nt = tix % nnt;
#pragma unroll
            for (int i = 0; i < 4; ++i) P[(long long)(m * 16 + 4 * grp + i) * kp + nt * 16 + col] = acc[j][i];
        }
    }
}

// out[e] = sum_b part[b][e] (fixed order), e < n.
__global__ void k_sum_blocks(const float *__restrict__ part, int nblk, long long n, float *__restrict__ out)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(long long)b * n + e];
    out[e] = s;
}

// ---------------------------------------------------------------- element-wise parts
__global__ void k_silu_bwd(const float *__restrict__ dA, const float *__restrict__ Y, float *__restrict__ dY,
                           long long n)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dY[e] = dA[e] * silu_grad(Y[e]);
}

// 2x2x2 average pooling: out (L/2)^3 from in L^3, per (batch, channel) plane set.
__global__ void k_pool(const float *__restrict__ in, float *__restrict__ out, int L, long long n_out)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_out) return;
    const int h = L / 2;
    const long long vo = (long long)h * h * h, vi = (long long)L * L * L;
    const long long bc = e / vo, r = e % vo;
    const int x = (int)(r % h), y = (int)((r / h) % h), z = (int)(r / ((long long)h * h));
    const float *p = in + bc * vi;
    float s = 0.0f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) s += p[(2 * x + dx) + (long long)L * ((2 * y + dy) + (long long)L * (2 * z + dz))];
    out[e] = 0.125f * s;
}

// gradient of the pooling: din[fine] (+)= dout[coarse] / 8
__global__ void k_pool_bwd(const float *__restrict__ dout, float *__restrict__ din, int L, long long n_in, int add)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_in) return;
    const int h = L / 2;
    const long long vo = (long long)h * h * h, vi = (long long)L * L * L;
    const long long bc = e / vi, r = e % vi;
    const int x = (int)(r % L), y = (int)((r / L) % L), z = (int)(r / ((long long)L * L));
    const float g = 0.125f * dout[bc * vo + (x / 2) + (long long)h * ((y / 2) + (long long)h * (z / 2))];
    din[e] = add ? din[e] + g : g;
}

// nearest 2x upsampling: out L^3 from in (L/2)^3
__global__ void k_up(const float *__restrict__ in, float *__restrict__ out, int L, long long n_out)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_out) return;
    const int h = L / 2;
    const long long vo = (long long)L * L * L, vi = (long long)h * h * h;
    const long long bc = e / vo, r = e % vo;
    const int x = (int)(r % L), y = (int)((r / L) % L), z = (int)(r / ((long long)L * L));
    out[e] = in[bc * vi + (x / 2) + (long long)h * ((y / 2) + (long long)h * (z / 2))];
}

// gradient of the upsampling: dcoarse = sum of the 8 fine gradients
__global__ void k_up_bwd(const float *__restrict__ dout, float *__restrict__ din, int L, long long n_in)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_in) return;
    const int h = L / 2;
    const long long vo = (long long)L * L * L, vi = (long long)h * h * h;
    const long long bc = e / vi, r = e % vi;
    const int x = (int)(r % h), y = (int)((r / h) % h), z = (int)(r / ((long long)h * h));
    const float *p = dout + bc * vo;
    float s = 0.0f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) s += p[(2 * x + dx) + (long long)L * ((2 * y + dy) + (long long)L * (2 * z + dz))];
    din[e] = s;
}

// c = a + b; with add_to: c += a
__global__ void k_add(const float *__restrict__ a, const float *__restrict__ b, float *__restrict__ c, long long n)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) c[e] = a[e] + (b ? b[e] : c[e]);
}

// per-channel sum over batch and sites: out[c] = sum_{b,x} g[b][c][x] (one block per channel)
__global__ __launch_bounds__(256) void k_channel_sum(const float *__restrict__ g, int B, int C, long long V,
                                                     float *__restrict__ out)
{
    const int c = blockIdx.x;
    double s = 0.0;
    for (int b = 0; b < B; ++b)
        for (long long x = threadIdx.x; x < V; x += 256) s += g[((long long)b * C + c) * V + x];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = (float)red[0];
}

// squared error: per-block partial sums of (p - t)^2 and dp = 2 (p - t) / count
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ p, const float *__restrict__ t,
                                             float *__restrict__ dp, long long n, float inv_count,
                                             double *__restrict__ part)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (e < n) {
        const float d = p[e] - t[e];
        v = (double)d * d;
        if (dp) dp[e] = 2.0f * d * inv_count;
    }
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam step on the FP32 master parameters.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    w[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
}

// BF16 matrix-core rows of one layer from its FP32 weights W[co][ci][27]:
//   fwd: Wm[o][k cip + c] = W[o][c][k]
//   dgrad (transposed, flipped): Wt[c][k cop' + o] = W[o][c][26 - k]  (cop' = co rounded up to 8)
__global__ void k_stage_weights(const float *__restrict__ W, int co, int ci, int cip, int kp, int cop_rows,
                                __bf16 *__restrict__ Wm, int cip_t, int kp_t, int cop_rows_t,
                                __bf16 *__restrict__ Wt)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nf = (long long)cop_rows * kp, nt = (long long)cop_rows_t * kp_t;
    if (e < nf) {
        const int o = (int)(e / kp), kk = (int)(e % kp);
        const int k = kk / cip, c = kk % cip;
        float v = 0.0f;
        if (o < co && k < 27 && c < ci) v = W[((long long)o * ci + c) * 27 + k];
        Wm[e] = (__bf16)v;
    } else if (e < nf + nt) {
        const long long f = e - nf;
        const int c = (int)(f / kp_t), kk = (int)(f % kp_t);
        const int k = kk / cip_t, o = kk % cip_t;
        float v = 0.0f;
        if (c < ci && k < 27 && o < co) v = W[((long long)o * ci + c) * 27 + (26 - k)];
        Wt[f] = (__bf16)v;
    }
}

// master-layout gradient dW[o][c][k] from the matrix-core layout dWm[o][k cip + c]
__global__ void k_unstage_grad(const float *__restrict__ dWm, int co, int ci, int cip, int kp,
                               float *__restrict__ dW)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)co * ci * 27;
    if (e >= n) return;
    const int k = (int)(e % 27), c = (int)((e / 27) % ci), o = (int)(e / (27LL * ci));
    dW[e] = dWm[(long long)o * kp + k * cip + c];
}

// Warm start from the network's prediction p (FP32, 2 polymer channels):
//   mode 0: w_I = p_I;  mode 1: w_I += p_I - p_prev_I
__global__ void k_warm_from_net(double *__restrict__ w, const float *__restrict__ p,
                                const float *__restrict__ p_prev, long long V, int mode)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * V) return;
    if (mode == 0) w[e] = (double)p[e];
    else w[e] += (double)p[e] - (double)p_prev[e];
}

// x[b][c][v] = (x - shift[c]) * scale[c]  (input normalisation of the network)
__global__ void k_affine(float *__restrict__ x, int C, long long V, long long n, const float *__restrict__ shift,
                         const float *__restrict__ scale)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int c = (int)((e / V) % C);
    x[e] = (x[e] - shift[c]) * scale[c];
}

// float <-> double copies
__global__ void k_f64_to_f32(const double *__restrict__ a, float *__restrict__ b, long long n)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) b[e] = (float)a[e];
}

// ---------------------------------------------------------------- launchers
static inline unsigned nb(long long n, int t) { return (unsigned)((n + t - 1) / t); }

void net_conv_fwd(hipStream_t s, const float *X, int B, int ci, int cip, const __bf16 *Wm, int kp, int co, int cop,
                  const float *bias, float *Y, float *A, int L)
{
    const int tx = (L + TX - 1) / TX, ty = (L + TY - 1) / TY, tz = (L + TZ - 1) / TZ;
    const int tps = tx * ty * tz;
    const size_t lds = (size_t)HS * cip * sizeof(__bf16);
    hipLaunchKernelGGL(k_conv_fwd, dim3(B * tps), dim3(256), lds, s, X, ci, cip, Wm, kp, co, cop, bias, Y, A, L, tx,
                       ty, tps);
}

// number of site slices of the weight gradient (partials buffer: slices x cop x kp floats)
int net_wgrad_blocks(int B, int L)
{
    const int tx = (L + TX - 1) / TX, ty = (L + TY - 1) / TY, tz = (L + TZ - 1) / TZ;
    const int n = B * tx * ty * tz;
    return n < 64 ? n : 64;
}

void net_conv_wgrad(hipStream_t s, const float *X, int B, int ci, int cip, const float *dY, int co, int cop, int kp,
                    int L, float *part, float *dWm)
{
    const int tx = (L + TX - 1) / TX, ty = (L + TY - 1) / TY, tz = (L + TZ - 1) / TZ;
    const int tps = tx * ty * tz, n_tiles = B * tps;
    const int slices = net_wgrad_blocks(B, L);
    const int ntiles = (cop / 16) * (kp / 16), groups = (ntiles + 15) / 16;
    const size_t lds = ((size_t)cip * HS + (size_t)cop * TS) * sizeof(__bf16);
    hipLaunchKernelGGL(k_conv_wgrad, dim3(groups * slices), dim3(256), lds, s, X, ci, cip, dY, co, cop, kp, L, tx,
                       ty, tps, n_tiles, groups, slices, part);
    const long long n = (long long)cop * kp;
    hipLaunchKernelGGL(k_sum_blocks, dim3(nb(n, 256)), dim3(256), 0, s, part, slices, n, dWm);
}

void net_silu_bwd(hipStream_t s, const float *dA, const float *Y, float *dY, long long n)
{
    hipLaunchKernelGGL(k_silu_bwd, dim3(nb(n, 256)), dim3(256), 0, s, dA, Y, dY, n);
}

void net_pool(hipStream_t s, const float *in, float *out, int L, long long n_out)
{
    hipLaunchKernelGGL(k_pool, dim3(nb(n_out, 256)), dim3(256), 0, s, in, out, L, n_out);
}

void net_pool_bwd(hipStream_t s, const float *dout, float *din, int L, long long n_in, int add)
{
    hipLaunchKernelGGL(k_pool_bwd, dim3(nb(n_in, 256)), dim3(256), 0, s, dout, din, L, n_in, add);
}

void net_up(hipStream_t s, const float *in, float *out, int L, long long n_out)
{
    hipLaunchKernelGGL(k_up, dim3(nb(n_out, 256)), dim3(256), 0, s, in, out, L, n_out);
}

void net_up_bwd(hipStream_t s, const float *dout, float *din, int L, long long n_in)
{
    hipLaunchKernelGGL(k_up_bwd, dim3(nb(n_in, 256)), dim3(256), 0, s, dout, din, L, n_in);
}

void net_add(hipStream_t s, const float *a, const float *b, float *c, long long n)
{
    hipLaunchKernelGGL(k_add, dim3(nb(n, 256)), dim3(256), 0, s, a, b, c, n);
}

void net_channel_sum(hipStream_t s, const float *g, int B, int C, long long V, float *out)
{
    hipLaunchKernelGGL(k_channel_sum, dim3(C), dim3(256), 0, s, g, B, C, V, out);
}

int net_mse(hipStream_t s, const float *p, const float *t, float *dp, long long n, float inv_count, double *part)
{
    const int blocks = (int)nb(n, 256);
    hipLaunchKernelGGL(k_mse, dim3(blocks), dim3(256), 0, s, p, t, dp, n, inv_count, part);
    return blocks;
}

void net_adam(hipStream_t s, float *w, const float *g, float *m, float *v, long long n, float lr, float b1, float b2,
              float eps, float c1, float c2)
{
    hipLaunchKernelGGL(k_adam, dim3(nb(n, 256)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

void net_stage_weights(hipStream_t s, const float *W, int co, int ci, int cip, int kp, int cop_rows, __bf16 *Wm,
                       int cip_t, int kp_t, int cop_rows_t, __bf16 *Wt)
{
    const long long n = (long long)cop_rows * kp + (long long)cop_rows_t * kp_t;
    hipLaunchKernelGGL(k_stage_weights, dim3(nb(n, 256)), dim3(256), 0, s, W, co, ci, cip, kp, cop_rows, Wm, cip_t,
                       kp_t, cop_rows_t, Wt);
}

void net_unstage_grad(hipStream_t s, const float *dWm, int co, int ci, int cip, int kp, float *dW)
{
    const long long n = (long long)co * ci * 27;
    hipLaunchKernelGGL(k_unstage_grad, dim3(nb(n, 256)), dim3(256), 0, s, dWm, co, ci, cip, kp, dW);
}

void net_warm_from_net(hipStream_t s, double *w, const float *p, const float *p_prev, long long V, int mode)
{
    hipLaunchKernelGGL(k_warm_from_net, dim3(nb(2 * V, 256)), dim3(256), 0, s, w, p, p_prev, V, mode);
}

void net_affine(hipStream_t s, float *x, int C, long long V, long long n, const float *shift, const float *scale)
{
    hipLaunchKernelGGL(k_affine, dim3(nb(n, 256)), dim3(256), 0, s, x, C, V, n, shift, scale);
}

void net_f64_to_f32(hipStream_t s, const double *a, float *b, long long n)
{
    hipLaunchKernelGGL(k_f64_to_f32, dim3(nb(n, 256)), dim3(256), 0, s, a, b, n);
}

}  // namespace hsf
