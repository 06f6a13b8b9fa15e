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
#include <algorithm>
#include <math.h>

#include "device_common.h"
#include "net_internal.h"

namespace hsf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
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
// Y[b][co][x] = bias[co] + sum_{ci,k} W[co][ci][k] X[b][ci][x + off_k], written as
// ConvOut asks (pre-activation, FP32 activation, packed BF16 activation).  The input
// tile with a one-site halo is staged in LDS as BF16 16-byte units of 8 channels,
// unit-major: xs[cip / 8][halo site][8].  A B operand read takes one unit of 16
// consecutive sites, i.e. 16 consecutive units: no two lanes of a 16-lane group share
// an LDS bank, whatever cip is (site-major rows of cip >= 16 channels would put sites
// 8 apart on the same banks).  The weights follow in slabs of kSlab K chunks (32 rows
// of K each), [cop][kSlab * 32 + 8] (the 8 extra columns stagger the rows over the LDS
// banks), so the K loop reads only LDS; the next slab's loads are in flight while the
// current one is multiplied.  Small slabs keep a 16x8x4 block of a 16-channel layer
// under 40 KB of LDS, four blocks per CU.
// The weight gradient works on TX x TY x TZ tiles (128 sites) staged channel-major.
constexpr int TX = 8, TY = 4, TZ = 4, TS = TX * TY * TZ;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HS = HX * HY * HZ;
constexpr int kSlab = 4;
constexpr int kSlabRow = kSlab * 32 + 8;

// periodic index for -L <= v < 2L (boxes at least one tile wide), general otherwise
__device__ __forceinline__ int wrap_tile(int v, int L, bool small)
{
    if (small) return wrapL(v, L);
    return v < 0 ? v + L : (v >= L ? v - L : v);
}


// Value of input channel c of sample b at site (gx, gy, gz) of the convolution's
// L^3 box, read through the input's composition (ConvIn): the tensor itself, the sum
// of two tensors (decoder skip), the nearest 2x upsampling of a tensor on the
// (L/2)^3 box, or the 2x2x2 average of a tensor on the (2L)^3 box (summed in the
// order dz, dy, dx, as the pooling of the backward pass assumes).
__device__ __forceinline__ float conv_input(const ConvIn &in, int b, int c, int ci, int gx, int gy, int gz, int L)
{
    if (in.mode == CONV_IN_UP) {
        const int h = L >> 1;
        const long long vh = (long long)h * h * h;
        return in.x1[((long long)b * ci + c) * vh + (gx >> 1) + (long long)h * ((gy >> 1) + (long long)h * (gz >> 1))];
    }
    if (in.mode == CONV_IN_POOL) {
        const int f = L << 1;
        const long long vf = (long long)f * f * f;
        const float *p = in.x1 + ((long long)b * ci + c) * vf;
        float s = 0.0f;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx)
                    s += p[(2 * gx + dx) + (long long)f * ((2 * gy + dy) + (long long)f * (2 * gz + dz))];
        return 0.125f * s;
    }
    const long long V = (long long)L * L * L;
    const long long e = ((long long)b * ci + c) * V + gx + (long long)L * (gy + (long long)L * gz);
    return in.mode == CONV_IN_ADD ? in.x1[e] + in.x2[e] : in.x1[e];
}

// Input rows of a TX x TY x TZ tile for the weight gradient, in LDS as BF16 in three
// x-shifted copies: xr[d][c][hz][hy][8] holds, for d = dx + 1, the input at x = x0 +
// dx + 0..7 of halo row (hy, hz) and channel c (channels ci..cip-1 zero; the channel
// pitch kWgChan pads 6 x 6 x 8 by 8 so the 16 lanes of a B operand read, 16 channels of
// one row, fall on distinct banks).  Every B operand of the K loop (8 consecutive
// sites of one channel at one tap) is then one aligned 16-byte read.
constexpr int kWgRows = (TZ + 2) * (TY + 2);   // halo rows of a tile
constexpr int kWgChan = kWgRows * TX + 8;      // channel pitch of a copy (elements)
constexpr int kWgYPitch = TS + 8;               // row pitch of the staged dY tile (odd in 16-byte units)
__device__ __forceinline__ void stage_rows3(const ConvIn &in, int b, int ci, int cip, int L, int x0, int y0, int z0,
                                            __bf16 *xr)
{
    // a work item is one value (halo position q of a row; consecutive items are
    // consecutive x, so a wave's loads are contiguous), stored into each copy that holds
    // it; eight values per thread in flight at once
    const bool small = L < TX;
    const int total = cip * kWgRows * (TX + 2);
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * 256;
            const int q = e % (TX + 2), r = e / (TX + 2), c = r / kWgRows, row = r % kWgRows;
            const int hz = row / HY, hy = row % HY;
            v[u] = 0.0f;
            if (e < total && c < ci)
                v[u] = conv_input(in, b, c, ci, wrap_tile(x0 + q - 1, L, small), wrap_tile(y0 + hy - 1, L, small),
                                  wrap_tile(z0 + hz - 1, L, small), L);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * 256;
            if (e >= total) continue;
            const int q = e % (TX + 2), r = e / (TX + 2), c = r / kWgRows, row = r % kWgRows;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int x = q - d;   // position of this value in copy d
                if (x >= 0 && x < TX) xr[(d * cip + c) * kWgChan + row * TX + x] = (__bf16)v[u];
            }
        }
    }
}

// A BX x BY x BZ tile with its one-site halo, unit-major xs[cip / 8][h][8] (forward): a
// work item is one halo site and eight consecutive channels, written to LDS as one
// 16-byte unit; two items (16 loads) per thread are in flight at once.
template <int BX, int BY, int BZ>
__device__ __forceinline__ void stage_halo_sm(const ConvIn &in, int b, int ci, int cip, int L, int x0, int y0,
                                              int z0, __bf16 *xs)
{
    constexpr int GX = BX + 2, GY = BY + 2, GS = GX * GY * (BZ + 2);
    constexpr int BMAX = BX > BY ? (BX > BZ ? BX : BZ) : (BY > BZ ? BY : BZ);
    const bool small = L < BMAX;
    const int oct = cip / 8, total = GS * oct;
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * 2) {
        float v[2][8];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = e0 + u * 256;
            const int c8 = e % oct, h = e / oct;
            const bool ok = e < total;
            const int hx = h % GX, hy = (h / GX) % GY, hz = h / (GX * GY);
            const int gx = wrap_tile(x0 + hx - 1, L, small), gy = wrap_tile(y0 + hy - 1, L, small),
                      gz = wrap_tile(z0 + hz - 1, L, small);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int c = c8 * 8 + j;
                v[u][j] = 0.0f;
                if (ok && c < ci) {
                    v[u][j] = conv_input(in, b, c, ci, gx, gy, gz, L);
                    if (in.shift) v[u][j] = (v[u][j] - in.shift[c]) * in.scale[c];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = e0 + u * 256;
            if (e < total) {
                bf16x8 pk;
#pragma unroll
                for (int j = 0; j < 8; ++j) pk[j] = (__bf16)v[u][j];
                *reinterpret_cast<bf16x8 *>(xs + ((e % oct) * GS + e / oct) * 8) = pk;
            }
        }
    }
}

// Row-vector staging of the same tile: aligned float4 loads of 4 consecutive x sites
// per channel, for plain and summed inputs on boxes at least a tile wide with L a
// multiple of 4 (three times fewer load instructions than one site per load).
typedef float floatv4 __attribute__((ext_vector_type(4)));
template <int BX, int BY, int BZ>
__device__ __forceinline__ void stage_halo_rows(const ConvIn &in, int b, int ci, int cip, int L, int x0, int y0,
                                                int z0, __bf16 *xs)
{
    constexpr int GX = BX + 2, GY = BY + 2, GZ = BZ + 2, GS = GX * GY * GZ;
    constexpr int NG = (BX + 8) / 4;   // float4 groups covering x in [x0 - 4, x0 + BX + 4)
    const int oct = cip / 8, total = GY * GZ * NG * oct;
    const long long V = (long long)L * L * L;
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * 2) {
        floatv4 v[2][8];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = e0 + u * 256;
            const bool ok = e < total;
            const int c8 = e % oct, r = e / oct;
            const int g = r % NG, row = r / NG;
            const int hy = row % GY, hz = row / GY;
            int xb = x0 - 4 + 4 * g;   // a multiple of 4; wraps as a whole group
            xb = xb < 0 ? xb + L : (xb >= L ? xb - L : xb);
            const int gy = wrap_tile(y0 + hy - 1, L, false), gz = wrap_tile(z0 + hz - 1, L, false);
            const long long site = xb + (long long)L * (gy + (long long)L * gz);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int c = c8 * 8 + j;
                v[u][j] = floatv4{0.f, 0.f, 0.f, 0.f};
                if (ok && c < ci) {
                    const long long a = ((long long)b * ci + c) * V + site;
                    v[u][j] = *reinterpret_cast<const floatv4 *>(in.x1 + a);
                    if (in.mode == CONV_IN_ADD) v[u][j] += *reinterpret_cast<const floatv4 *>(in.x2 + a);
                    if (in.shift) v[u][j] = (v[u][j] - in.shift[c]) * in.scale[c];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = e0 + u * 256;
            if (e < total) {
                const int c8 = e % oct, r = e / oct;
                const int g = r % NG, row = r / NG;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int hx = 4 * g + q - 3;   // halo x position of this site
                    if (hx >= 0 && hx < GX) {
                        bf16x8 pk;
#pragma unroll
                        for (int j = 0; j < 8; ++j) pk[j] = (__bf16)v[u][j][q];
                        *reinterpret_cast<bf16x8 *>(xs + (c8 * GS + row * GX + hx) * 8) = pk;
                    }
                }
            }
        }
    }
}

// The same tile from a packed BF16 input (CONV_IN_PACKED): halo unit e (site e / (cip /
// 8), channels 8 (e % (cip / 8)) + 0..7) is one 16-byte copy from global memory (site
// after site, so the loads are contiguous) to its unit-major LDS place; eight copies
// per thread are in flight at once.
template <int BX, int BY, int BZ>
__device__ __forceinline__ void stage_halo_packed(const __bf16 *__restrict__ xp, int b, int cip, int L, int x0,
                                                  int y0, int z0, __bf16 *xs)
{
    constexpr int GX = BX + 2, GY = BY + 2, GS = GX * GY * (BZ + 2);
    constexpr int BMAX = BX > BY ? (BX > BZ ? BX : BZ) : (BY > BZ ? BY : BZ);
    constexpr int U = 8;
    const bool small = L < BMAX;
    const int oct = cip / 8, total = GS * oct;
    const __bf16 *base = xp + (long long)b * L * L * L * cip;
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * U) {
        bf16x8 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * 256;
            if (e < total) {
                const int c8 = e % oct, h = e / oct;
                const int hx = h % GX, hy = (h / GX) % GY, hz = h / (GX * GY);
                const int gx = wrap_tile(x0 + hx - 1, L, small), gy = wrap_tile(y0 + hy - 1, L, small),
                          gz = wrap_tile(z0 + hz - 1, L, small);
                const long long site = gx + (long long)L * (gy + (long long)L * gz);
                v[u] = *reinterpret_cast<const bf16x8 *>(base + site * cip + 8 * c8);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * 256;
            if (e < total) *reinterpret_cast<bf16x8 *>(xs + ((e % oct) * GS + e / oct) * 8) = v[u];
        }
    }
}

constexpr int kMaxKGroups = 27 * 32 / 8 + 4;   // K rows / 8 for cip <= 32, rounded up to 32 rows

template <int BX, int BY, int BZ>
constexpr size_t conv_fwd_lds_t(int cip, int cop)
{
    return (size_t)((BX + 2) * (BY + 2) * (BZ + 2) * cip + cop * kSlabRow) * sizeof(__bf16) +
           kMaxKGroups * sizeof(int);
}

// Block: a BX x BY x BZ tile of one sample; its 16-site MFMA column tiles are dealt to
// the four waves (NTW each), each with NM = cop / 16 (1 or 2) 16-channel output tiles.
template <int BX, int BY, int BZ, int NM>
__global__ __launch_bounds__(256) void k_conv_fwd(ConvIn in, int ci, int cip, const __bf16 *__restrict__ Wm, int kp,
                                                   int co, int cop, const float *__restrict__ bias, ConvOut out, int L,
                                                   int tiles_x, int tiles_y, int tiles_per_sample)
{
    constexpr int BS = BX * BY * BZ, GX = BX + 2, GY = BY + 2, GS = GX * GY * (BZ + 2);
    constexpr int NTW = BS / 64;   // column tiles per wave
    constexpr int NPRE = (NM * 16 * kSlab * 4 + 255) / 256;   // weight vectors per thread and slab
    static_assert(BS % 64 == 0 && BX % 8 == 0, "tile shape");
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16 *xs = reinterpret_cast<__bf16 *>(smem);   // [cip / 8][GS][8]
    __bf16 *ws = xs + GS * cip;                       // [cop][kSlabRow]
    int *koff = reinterpret_cast<int *>(ws + cop * kSlabRow);   // [kp / 8]
    const int bid = plan_block();   // neighbouring tiles on one XCD
    const int b = bid / tiles_per_sample;
    int t = bid % tiles_per_sample;
    const int x0 = (t % tiles_x) * BX;
    t /= tiles_x;
    const int y0 = (t % tiles_y) * BY;
    const int z0 = (t / tiles_y) * BZ;
    const long long V = (long long)L * L * L;
    // weight slab k0 (rows of kp, k0 .. k0 + kSlab * 32) through registers: load(k0)
    // issues the loads, store(k0) writes what arrived to LDS
    bf16x8 wv[NPRE];
    auto slab_vectors = [&](int k0, int &vec_per_row) {
        vec_per_row = min(kSlab * 32, kp - k0) / 8;
        return cop * vec_per_row;
    };
    auto load_slab = [&](int k0) {
        int vpr;
        const int nvec = slab_vectors(k0, vpr);
#pragma unroll
        for (int u = 0; u < NPRE; ++u) {
            const int e = threadIdx.x + u * 256;
            if (e < nvec) {
                const int r = e / vpr, v8 = e - r * vpr;
                wv[u] = *reinterpret_cast<const bf16x8 *>(Wm + (long long)r * kp + k0 + 8 * v8);
            }
        }
    };
    auto store_slab = [&](int k0) {
        int vpr;
        const int nvec = slab_vectors(k0, vpr);
#pragma unroll
        for (int u = 0; u < NPRE; ++u) {
            const int e = threadIdx.x + u * 256;
            if (e < nvec) {
                const int r = e / vpr, v8 = e - r * vpr;
                *reinterpret_cast<bf16x8 *>(ws + r * kSlabRow + 8 * v8) = wv[u];
            }
        }
    };
    load_slab(0);   // in flight with the tile's loads
    // LDS element offset, relative to 8 times a site's halo position, of each group of
    // eight K rows (tap k, channels c0..c0+7: unit c0 / 8 of the tap's neighbour);
    // padding rows point at the centre tap (zero weights there)
    for (int g = threadIdx.x; g < kp / 8; g += 256) {
        int k = (8 * g) / cip;
        const int c0 = 8 * g - k * cip;
        if (k > 26) k = 13;
        koff[g] = ((((k / 9) - 1) * GX * GY + (((k / 3) % 3) - 1) * GX + ((k % 3) - 1)) + (c0 / 8) * GS) * 8;
    }
    if (in.mode == CONV_IN_PACKED)
        stage_halo_packed<BX, BY, BZ>(in.xp, b, cip, L, x0, y0, z0, xs);
    else if ((in.mode == CONV_IN_PLAIN || in.mode == CONV_IN_ADD) && L % 4 == 0 && L >= BX && L >= BY && L >= BZ)
        stage_halo_rows<BX, BY, BZ>(in, b, ci, cip, L, x0, y0, z0, xs);
    else
        stage_halo_sm<BX, BY, BZ>(in, b, ci, cip, L, x0, y0, z0, xs);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane >> 4, col = lane & 15;
    floatx4 acc[NTW][NM];
#pragma unroll
    for (int q = 0; q < NTW; ++q)
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[q][m] = floatx4{0.f, 0.f, 0.f, 0.f};
    // this lane's sites (column of the B operand): LDS element offsets of their halo
    // positions
    int hbase[NTW];
#pragma unroll
    for (int q = 0; q < NTW; ++q) {
        const int n = (wave * NTW + q) * 16 + col;
        const int tx = n % BX, ty = (n / BX) % BY, tz = n / (BX * BY);
        hbase[q] = ((tz + 1) * GX * GY + (ty + 1) * GX + (tx + 1)) * 8;
    }
    for (int k0 = 0; k0 < kp; k0 += kSlab * 32) {
        const int klen = min(kSlab * 32, kp - k0);
        __syncthreads();   // previous slab consumed (and, the first time, the halo staged)
        store_slab(k0);
        if (k0 + kSlab * 32 < kp) load_slab(k0 + kSlab * 32);
        __syncthreads();
        const __bf16 *wa = ws + col * kSlabRow + 8 * grp;
        const int *kg = koff + k0 / 8 + grp;
        for (int kc = 0; kc < klen; kc += 32) {
            const int off = kg[kc / 8];
            bf16x8 a[NM];
#pragma unroll
            for (int m = 0; m < NM; ++m) a[m] = *reinterpret_cast<const bf16x8 *>(wa + m * 16 * kSlabRow + kc);
#pragma unroll
            for (int q = 0; q < NTW; ++q) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(xs + hbase[q] + off);
#pragma unroll
                for (int m = 0; m < NM; ++m)
                    acc[q][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bv, acc[q][m], 0, 0, 0);
            }
        }
    }
    // epilogue: lane holds rows 4 grp + i of each M tile, column = its site
    float *Yb = out.Y ? out.Y + (long long)b * co * V : nullptr;
    float *Ab = out.A ? out.A + (long long)b * co * V : nullptr;
    const int cpk = (co + 7) & ~7;   // channel stride of the packed activation
    __bf16 *Pb = out.Ap ? out.Ap + (long long)b * V * cpk : nullptr;
#pragma unroll
    for (int q = 0; q < NTW; ++q) {
        const int n = (wave * NTW + q) * 16 + col;
        const int tx = n % BX, ty = (n / BX) % BY, tz = n / (BX * BY);
        const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
        if (gx >= L || gy >= L || gz >= L) continue;
        const long long site = gx + (long long)L * (gy + (long long)L * gz);
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const int o0 = m * 16 + 4 * grp;
            if (Pb && o0 < cpk) {   // four consecutive channels of the site: one 8-byte store
                bf16x4 pk;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int o = o0 + i;
                    pk[i] = (__bf16)(o < co ? silu(acc[q][m][i] + (bias ? bias[o] : 0.0f)) : 0.0f);
                }
                *reinterpret_cast<bf16x4 *>(Pb + site * cpk + o0) = pk;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = o0 + i;
                if (o >= co) continue;
                float y = acc[q][m][i] + (bias ? bias[o] : 0.0f);
                if (Ab) Ab[(long long)o * V + site] = silu(y);
                if (out.shift) y = (y - out.shift[o]) * out.scale[o];
                if (Yb) Yb[(long long)o * V + site] = y;
            }
        }
    }
}

// ---------------------------------------------------------------- weight gradient
// dW[co][k cip + ci] = sum_b sum_x dY[b][co][x] X[b][ci][x + off_k], as the GEMM
// C (cop x kp) = A (cop x sites) B (sites x kp).  Block (g, sp): the up to 4 x
// WG_TILES_PER_WAVE C tiles of group g (WG_TILES_PER_WAVE per wave, accumulated in
// registers) over the site tiles sp, sp + nsp, ... (K chunks of 32 sites = 4 x-rows of
// 8).  A operands (dY, [cop][TS]) are shared by a wave's tiles; B operands come from
// the shifted row copies (one 16-byte read each).  Partial C per site slice goes to
// `part` [sp][cop][kp] and is summed in a fixed order by k_sum_blocks.
constexpr int WG_TILES_PER_WAVE = 8;
constexpr int WG_TILES_PER_BLOCK = 4 * WG_TILES_PER_WAVE;

__global__ __launch_bounds__(256) void k_conv_wgrad(ConvIn in, int ci, int cip,
                                                     const float *__restrict__ dY, int co, int cop, int kp,
                                                     int L, int tiles_x, int tiles_y, int tiles_per_sample,
                                                     int n_tiles, int n_groups, int n_slices,
                                                     float *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16 *xr = reinterpret_cast<__bf16 *>(smem);        // [3][cip][kWgChan]
    __bf16 *ys = xr + (size_t)3 * cip * kWgChan;         // [cop][kWgYPitch]
    const int g = blockIdx.x % n_groups, sp = blockIdx.x / n_groups;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane >> 4, col = lane & 15;
    const int nnt = kp / 16, ntiles = (cop / 16) * nnt;
    const long long V = (long long)L * L * L;
    // this lane's B column of each of the wave's tiles: LDS offset of the row copy at the
    // tile's centre row (-1 for the zero padding rows of K) and the tile's M tile
    int boff[WG_TILES_PER_WAVE], mt[WG_TILES_PER_WAVE];
#pragma unroll
    for (int j = 0; j < WG_TILES_PER_WAVE; ++j) {
        const int tix = g * WG_TILES_PER_BLOCK + wave * WG_TILES_PER_WAVE + j;
        const int nt = tix % nnt, kk = nt * 16 + col, k = kk / cip, c = kk - k * cip;
        mt[j] = tix / nnt;
        boff[j] = -1;
        if (tix < ntiles && k <= 26) {
            const int dx = (k % 3) - 1, dy = ((k / 3) % 3) - 1, dz = (k / 9) - 1;
            boff[j] = ((dx + 1) * cip + c) * kWgChan + ((1 + dz) * HY + (1 + dy)) * TX;
        }
    }
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
        stage_rows3(in, b, ci, cip, L, x0, y0, z0, xr);
        for (int e0 = threadIdx.x; e0 < TS * cop; e0 += 256 * 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 256;
                const int n = e % TS, o = e / TS;
                const int tx = n % TX, ty = (n / TX) % TY, tz = n / (TX * TY);
                const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
                v[u] = 0.0f;
                if (e < TS * cop && o < co && gx < L && gy < L && gz < L)   // sites outside the box add nothing
                    v[u] = dY[((long long)b * co + o) * V + gx + (long long)L * (gy + (long long)L * gz)];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 256;
                if (e < TS * cop) ys[(e / TS) * kWgYPitch + e % TS] = (__bf16)v[u];
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int kc = 0; kc < TS; kc += 32) {
            // 8 consecutive sites of this lane group: one x-row of the tile
            const int s0 = kc + 8 * grp;
            const int ty = (s0 / TX) % TY, tz = s0 / (TX * TY);
            const int roff = (tz * HY + ty) * TX;
            const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(ys + col * kWgYPitch + s0);
            bf16x8 a1 = a0;
            if (cop > 16) a1 = *reinterpret_cast<const bf16x8 *>(ys + (16 + col) * kWgYPitch + s0);
#pragma unroll
            for (int j = 0; j < WG_TILES_PER_WAVE; ++j) {
                const int tix = g * WG_TILES_PER_BLOCK + wave * WG_TILES_PER_WAVE + j;
                if (tix < ntiles) {
                    bf16x8 bv;
                    if (boff[j] < 0) {
#pragma unroll
                        for (int q = 0; q < 8; ++q) bv[q] = (__bf16)0.0f;
                    } else {
                        bv = *reinterpret_cast<const bf16x8 *>(xr + boff[j] + roff);
                    }
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mt[j] ? a1 : a0, bv, acc[j], 0, 0, 0);
                }
            }
        }
    }
    float *P = part + (long long)sp * cop * kp;
#pragma unroll
    for (int j = 0; j < WG_TILES_PER_WAVE; ++j) {
        const int tix = g * WG_TILES_PER_BLOCK + wave * WG_TILES_PER_WAVE + j;
        if (tix < ntiles) {
            const int m = tix / nnt, nt = tix % nnt;
#pragma unroll
            for (int i = 0; i < 4; ++i) P[(long long)(m * 16 + 4 * grp + i) * kp + nt * 16 + col] = acc[j][i];
        }
    }
}

// out[e] = sum_b part[b][e], e < n, in a fixed order: thread (j, e) sums the partials
// b = j, j + 32, ... of element e; the 32 sums are then added in order j = 0..31.  A
// block covers 8 elements (32-byte rows of consecutive elements per partial).
__global__ __launch_bounds__(256) void k_sum_blocks(const float *__restrict__ part, int nblk, long long n,
                                                    float *__restrict__ out)
{
    __shared__ float red[32][8];
    const int el = threadIdx.x & 7, j = threadIdx.x >> 3;
    const long long e = (long long)blockIdx.x * 8 + el;
    float s = 0.0f;
    if (e < n)
        for (int b = j; b < nblk; b += 32) s += part[(long long)b * n + e];
    red[j][el] = s;
    __syncthreads();
    if (j == 0 && e < n) {
        float t = red[0][el];
#pragma unroll
        for (int q = 1; q < 32; ++q) t += red[q][el];
        out[e] = t;
    }
}

// ---------------------------------------------------------------- element-wise parts
__global__ void k_silu_bwd(const float *__restrict__ dA, const float *__restrict__ Y, float *__restrict__ dY,
                           long long n)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dY[e] = dA[e] * silu_grad(Y[e]);
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

// gradient of the upsampling: dcoarse (+)= sum of the 8 fine gradients
__global__ void k_up_bwd(const float *__restrict__ dout, float *__restrict__ din, int L, long long n_in, int add)
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
    din[e] = add ? din[e] + s : s;
}

// dst = src, or dst += src
__global__ void k_accum(float *__restrict__ dst, const float *__restrict__ src, long long n, int add)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = add ? dst[e] + src[e] : src[e];
}

// Per-channel sum over batch and sites, out[c] = sum_{b,x} g[b][c][x], in two fixed-order
// stages: block (c, j) sums slice j of the B V values of channel c into part[c][j];
// k_channel_final adds the slices in order.
constexpr int kChanSlices = 64;

__global__ __launch_bounds__(256) void k_channel_partial(const float *__restrict__ g, int B, int C, long long V,
                                                         double *__restrict__ part)
{
    const int c = blockIdx.x / kChanSlices, j = blockIdx.x % kChanSlices;
    const long long n = (long long)B * V, per = (n + kChanSlices - 1) / kChanSlices;
    const long long lo = j * per, hi = min(n, lo + per);
    double s = 0.0;
    for (long long e = lo + threadIdx.x; e < hi; e += 256) {
        const long long b = e / V, x = e - b * V;
        s += g[(b * C + c) * V + x];
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_channel_final(const double *__restrict__ part, int C, float *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double s = 0.0;
    for (int j = 0; j < kChanSlices; ++j) s += part[c * kChanSlices + j];
    out[c] = (float)s;
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
// ---------------------------------------------------------------- warm start
// Difference of densities used as the network's second input group:
//   mode 1: delta = phi - h0                (first difference)
//   mode 2: delta = phi - 2 h0 + h1         (second difference)
__device__ __forceinline__ double warm_delta(const double *phi, const double *h0, const double *h1, long long e,
                                             int mode)
{
    return mode == 2 ? (phi[e] - 2.0 * h0[e] + h1[e]) : (phi[e] - h0[e]);
}

// Per-block partial sums of delta^2 over the nsp x V values of one replica.
__global__ __launch_bounds__(256) void k_delta_sumsq(const double *__restrict__ phi, const double *__restrict__ h0,
                                                     const double *__restrict__ h1, long long n, int mode,
                                                     double *__restrict__ part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const double d = warm_delta(phi, h0, h1, e, mode);
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// rms = sqrt(sum of the partials / n), floored so that a zero difference divides safely.
__global__ __launch_bounds__(256) void k_delta_rms(const double *__restrict__ part, int nparts, long long n,
                                                   double *__restrict__ rms)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) rms[0] = fmax(sqrt(red[0] / (double)n), 1e-300);
}

// Network input of one replica ([channel][V] FP32):
//   mode 0: x = phi                                   (nsp channels)
//   mode 1, 2: x = (h0, delta / rms)                  (2 nsp channels)
__global__ void k_net_input(const double *__restrict__ phi, const double *__restrict__ h0,
                            const double *__restrict__ h1, long long n, int mode, const double *__restrict__ rms,
                            float *__restrict__ x)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    if (mode == 0) {
        x[e] = (float)phi[e];
        return;
    }
    x[e] = (float)h0[e];
    x[n + e] = (float)(warm_delta(phi, h0, h1, e, mode) / rms[0]);
}

// Apply the prediction p ([2][V]) to the polymer fields w ([2][V] of the replica):
//   mode 0: w = p;  mode 1: w += rms p;  mode 2: w += (wh0 - wh1) + rms p.
__global__ void k_warm_apply(double *__restrict__ w, const float *__restrict__ p, long long n, int mode,
                             const double *__restrict__ rms, const double *__restrict__ wh0,
                             const double *__restrict__ wh1)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    if (mode == 0) {
        w[e] = (double)p[e];
        return;
    }
    double v = w[e] + rms[0] * (double)p[e];
    if (mode == 2) v += wh0[e] - wh1[e];
    w[e] = v;
}

// Training target of one replica over the polymer channels (the first 2 V values of the
// field layout): mode 0, the fields themselves; modes 1 and 2, delta w / rms with delta as
// in warm_delta.
__global__ void k_net_target(const double *__restrict__ w, const double *__restrict__ w0,
                             const double *__restrict__ w1, long long n, int mode, const double *__restrict__ rms,
                             float *__restrict__ y)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = (float)(mode == 0 ? w[e] : warm_delta(w, w0, w1, e, mode) / rms[0]);
}

// Per-channel partial sums of x and x^2 over batch and sites: block (c, k) of a grid of
// C x nblk blocks covers every nblk-th chunk of 256 values of channel c.
__global__ __launch_bounds__(256) void k_channel_sums(const float *__restrict__ x, int batch, int C, long long V,
                                                      int nblk, double *__restrict__ part)
{
    const int c = blockIdx.x, k = blockIdx.y;
    __shared__ double r1[256], r2[256];
    double s1 = 0.0, s2 = 0.0;
    const long long n = (long long)batch * V;
    for (long long e = (long long)k * 256 + threadIdx.x; e < n; e += (long long)nblk * 256) {
        const long long b = e / V, i = e - b * V;
        const double v = (double)x[(b * C + c) * V + i];
        s1 += v;
        s2 += v * v;
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            r1[threadIdx.x] += r1[threadIdx.x + h];
            r2[threadIdx.x] += r2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * ((long long)c * nblk + k)] = r1[0];
        part[2 * ((long long)c * nblk + k) + 1] = r2[0];
    }
}

// out[2 c] = mean, out[2 c + 1] = root mean square of channel c (partials summed in order).
__global__ void k_channel_finish(const double *__restrict__ part, int C, int nblk, double count,
                                 double *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < nblk; ++k) {
        s1 += part[2 * ((long long)c * nblk + k)];
        s2 += part[2 * ((long long)c * nblk + k) + 1];
    }
    out[2 * c] = s1 / count;
    out[2 * c + 1] = sqrt(s2 / count);
}

// w += wh0 - wh1 (plain extrapolation of the fields)
__global__ void k_shift_fields(double *__restrict__ w, const double *__restrict__ wh0,
                               const double *__restrict__ wh1, long long n)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) w[e] += wh0[e] - wh1[e];
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


// ---------------------------------------------------------------- launchers
static inline unsigned nb(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// Largest dynamic LDS a block may use on the current device (queried once).
static size_t lds_limit()
{
    static size_t lim = 0;
    if (!lim) {
        int dev = 0, v = 0;
        lim = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            lim = std::min<size_t>((size_t)v, 65536);
    }
    return lim;
}

template <int BX, int BY, int BZ>
static void conv_fwd_launch(hipStream_t s, ConvIn in, int B, int ci, int cip, const __bf16 *Wm, int kp, int co,
                            int cop, const float *bias, ConvOut out, int L)
{
    const int tx = (L + BX - 1) / BX, ty = (L + BY - 1) / BY, tz = (L + BZ - 1) / BZ;
    const int tps = tx * ty * tz;
    const size_t lds = conv_fwd_lds_t<BX, BY, BZ>(cip, cop);
    if (cop == 16)
        hipLaunchKernelGGL((k_conv_fwd<BX, BY, BZ, 1>), dim3(B * tps), dim3(256), lds, s, in, ci, cip, Wm, kp, co, cop,
                           bias, out, L, tx, ty, tps);
    else
        hipLaunchKernelGGL((k_conv_fwd<BX, BY, BZ, 2>), dim3(B * tps), dim3(256), lds, s, in, ci, cip, Wm, kp, co, cop,
                           bias, out, L, tx, ty, tps);
}

// Tile per layer: the largest of 16x8x4, 8x8x4, 8x4x4 that the box fills, whose LDS
// (halo tile plus one weight slab) fits, and that still gives the launch at least
// kMinConvBlocks blocks; else 8x4x2.  Larger tiles re-read fewer halo sites and stage
// the weights for more sites; on the coarse levels of a U-Net (8^3, 16^3 boxes) they
// would leave a launch with a handful of blocks, each working through all of its sites
// in turn.  The tile does not change any result: every output sums its K chunks in the
// same order.
constexpr long long kMinConvBlocks = 256;

static long long conv_blocks(int B, int L, int bx, int by, int bz)
{
    return (long long)B * ((L + bx - 1) / bx) * ((L + by - 1) / by) * ((L + bz - 1) / bz);
}

void net_conv_fwd(hipStream_t s, ConvIn in, int B, int ci, int cip, const __bf16 *Wm, int kp, int co, int cop,
                  const float *bias, ConvOut out, int L)
{
    const size_t lim = lds_limit();
    if (L >= 16 && conv_fwd_lds_t<16, 8, 4>(cip, cop) <= lim && conv_blocks(B, L, 16, 8, 4) >= kMinConvBlocks)
        conv_fwd_launch<16, 8, 4>(s, in, B, ci, cip, Wm, kp, co, cop, bias, out, L);
    else if (L >= 8 && conv_fwd_lds_t<8, 8, 4>(cip, cop) <= lim && conv_blocks(B, L, 8, 8, 4) >= kMinConvBlocks)
        conv_fwd_launch<8, 8, 4>(s, in, B, ci, cip, Wm, kp, co, cop, bias, out, L);
    else if (conv_fwd_lds_t<8, 4, 4>(cip, cop) <= lim && conv_blocks(B, L, 8, 4, 4) >= kMinConvBlocks)
        conv_fwd_launch<8, 4, 4>(s, in, B, ci, cip, Wm, kp, co, cop, bias, out, L);
    else
        conv_fwd_launch<8, 4, 2>(s, in, B, ci, cip, Wm, kp, co, cop, bias, out, L);
}

// Site slices of the weight gradient: enough blocks (groups x slices, about 1024) to
// fill the chip, each covering at least one site tile.  The partials buffer holds
// slices x cop x kp floats.
int net_wgrad_slices(int B, int L, int cop, int kp)
{
    const int tx = (L + TX - 1) / TX, ty = (L + TY - 1) / TY, tz = (L + TZ - 1) / TZ;
    const int n_tiles = B * tx * ty * tz;
    const int groups = ((cop / 16) * (kp / 16) + WG_TILES_PER_BLOCK - 1) / WG_TILES_PER_BLOCK;
    const int want = std::max(1, 1024 / groups);
    return std::min(n_tiles, want);
}

void net_conv_wgrad(hipStream_t s, ConvIn in, int B, int ci, int cip, const float *dY, int co, int cop, int kp,
                    int L, float *part, float *dWm)
{
    const int tx = (L + TX - 1) / TX, ty = (L + TY - 1) / TY, tz = (L + TZ - 1) / TZ;
    const int tps = tx * ty * tz, n_tiles = B * tps;
    const int slices = net_wgrad_slices(B, L, cop, kp);
    const int ntiles = (cop / 16) * (kp / 16), groups = (ntiles + WG_TILES_PER_BLOCK - 1) / WG_TILES_PER_BLOCK;
    const size_t lds = ((size_t)3 * cip * kWgChan + (size_t)cop * kWgYPitch) * sizeof(__bf16);
    hipLaunchKernelGGL(k_conv_wgrad, dim3(groups * slices), dim3(256), lds, s, in, ci, cip, dY, co, cop, kp, L, tx,
                       ty, tps, n_tiles, groups, slices, part);
    const long long n = (long long)cop * kp;
    hipLaunchKernelGGL(k_sum_blocks, dim3(nb(n, 8)), dim3(256), 0, s, part, slices, n, dWm);
}

void net_silu_bwd(hipStream_t s, const float *dA, const float *Y, float *dY, long long n)
{
    hipLaunchKernelGGL(k_silu_bwd, dim3(nb(n, 256)), dim3(256), 0, s, dA, Y, dY, n);
}

void net_pool_bwd(hipStream_t s, const float *dout, float *din, int L, long long n_in, int add)
{
    hipLaunchKernelGGL(k_pool_bwd, dim3(nb(n_in, 256)), dim3(256), 0, s, dout, din, L, n_in, add);
}

void net_up_bwd(hipStream_t s, const float *dout, float *din, int L, long long n_in, int add)
{
    hipLaunchKernelGGL(k_up_bwd, dim3(nb(n_in, 256)), dim3(256), 0, s, dout, din, L, n_in, add);
}

void net_accum(hipStream_t s, float *dst, const float *src, long long n, int add)
{
    hipLaunchKernelGGL(k_accum, dim3(nb(n, 256)), dim3(256), 0, s, dst, src, n, add);
}

int net_channel_parts(int C) { return C * kChanSlices; }

void net_channel_sum(hipStream_t s, const float *g, int B, int C, long long V, double *part, float *out)
{
    hipLaunchKernelGGL(k_channel_partial, dim3(C * kChanSlices), dim3(256), 0, s, g, B, C, V, part);
    hipLaunchKernelGGL(k_channel_final, dim3(1), dim3(64), 0, s, part, C, out);
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

void net_warm_input(hipStream_t s, const double *phi, const double *h0, const double *h1, int nsp, long long V,
                    int mode, double *part, int max_parts, double *rms, float *x)
{
    const long long n = (long long)nsp * V;
    if (mode != 0) {
        const int nparts = (int)std::min<long long>(max_parts, std::max<long long>(1, nb(n, 256)));
        hipLaunchKernelGGL(k_delta_sumsq, dim3(nparts), dim3(256), 0, s, phi, h0, h1, n, mode, part);
        hipLaunchKernelGGL(k_delta_rms, dim3(1), dim3(256), 0, s, part, nparts, n, rms);
    }
    hipLaunchKernelGGL(k_net_input, dim3(nb(n, 256)), dim3(256), 0, s, phi, h0, h1, n, mode, rms, x);
}

void net_warm_apply(hipStream_t s, double *w, const float *p, long long V, int mode, const double *rms,
                    const double *wh0, const double *wh1)
{
    hipLaunchKernelGGL(k_warm_apply, dim3(nb(2 * V, 256)), dim3(256), 0, s, w, p, 2 * V, mode, rms, wh0, wh1);
}

void net_shift_fields(hipStream_t s, double *w, const double *wh0, const double *wh1, long long n)
{
    hipLaunchKernelGGL(k_shift_fields, dim3(nb(n, 256)), dim3(256), 0, s, w, wh0, wh1, n);
}

void net_sample(hipStream_t s, const double *phi, const double *phi0, const double *phi1, const double *w,
                const double *w0, const double *w1, int nsp, long long V, int mode, double *part, int max_parts,
                double *rms, float *x, float *y)
{
    net_warm_input(s, phi, phi0, phi1, nsp, V, mode, part, max_parts, rms, x);
    hipLaunchKernelGGL(k_net_target, dim3(nb(2 * V, 256)), dim3(256), 0, s, w, w0, w1, 2 * V, mode, rms, y);
}

void net_channel_moments(hipStream_t s, const float *x, int batch, int C, long long V, double *part, int nblk,
                         double *out)
{
    hipLaunchKernelGGL(k_channel_sums, dim3(C, nblk), dim3(256), 0, s, x, batch, C, V, nblk, part);
    hipLaunchKernelGGL(k_channel_finish, dim3(1), dim3(64), 0, s, part, C, nblk, (double)batch * (double)V, out);
}

void net_affine(hipStream_t s, float *x, int C, long long V, long long n, const float *shift, const float *scale)
{
    hipLaunchKernelGGL(k_affine, dim3(nb(n, 256)), dim3(256), 0, s, x, C, V, n, shift, scale);
}


}  // namespace hsf
