// prop_block.hip -- temporally blocked propagator sweeps (eq. 16-17).
//
// One launch advances K contour steps.  Each block owns a core tile of
// CX x CY x CZ sites and stages the propagator on the core plus a halo of K
// sites per side in LDS; level k (k = 1..K) applies the 27-point linkage
// stencil on the region that shrinks by one site per side per level, so the
// core after K levels is exact.  Every level writes its core to the global
// store G_s (forward) or adds G_s sigma[G+_{s+1}] into per-core accumulators
// (backward); the next launch starts from the stored core planes.  Halo sites
// are recomputed by neighbouring blocks (the price of fewer launches).
//
// Scaling: stored G_s = G_s / 2^(e_1+..+e_s), stored G+_s = G+_s 2^(e_1+..+e_{s-1}) /
// 2^(e_1+..+e_N): the same per-step power of two divides both sweeps, so every
// product G_s sigma[G+_{s+1}] carries one common factor that cancels in phi.
#include <hip/hip_ext.h>
#include <type_traits>

#include "device_common.h"
#include "prop_block.h"

namespace hsf {

template <typename real>
__device__ __forceinline__ real pow2_neg_b(int e)
{
    return (real)ldexp(1.0, -e);
}

__device__ __forceinline__ int wrapn(int v, int L)
{
    v %= L;
    return v < 0 ? v + L : v;
}

// Tile of this block: replica, core origin, and per-axis global offsets of the region.
template <int CX, int CY, int CZ, int K>
struct TileCtx {
    static constexpr int NX = CX + 2 * K, NY = CY + 2 * K, NZ = CZ + 2 * K;
    int r;
    int x0, y0, z0;
};

// Iterations of a kBlock-thread loop over the level-k region, and the region position
// of iteration `it` of this thread (false past the region's end).
template <int CX, int CY, int CZ, int K>
__host__ __device__ constexpr int region_iters(int k)
{
    return ((CX + 2 * (K - k)) * (CY + 2 * (K - k)) * (CZ + 2 * (K - k)) + kBlock - 1) / kBlock;
}

template <int CX, int CY, int CZ, int K>
__host__ __device__ constexpr int region_iters_total()
{
    int n = 0;
    for (int k = 1; k <= K; ++k) n += region_iters<CX, CY, CZ, K>(k);
    return n;
}

template <int CX, int CY, int CZ, int K>
__device__ __forceinline__ bool region_pos(int k, int it, int &px, int &py, int &pz)
{
    constexpr int NX = CX + 2 * K, NY = CY + 2 * K, NZ = CZ + 2 * K;
    const int mx = NX - 2 * k, my = NY - 2 * k, mz = NZ - 2 * k;
    const int t = (int)threadIdx.x + it * kBlock;
    if (t >= mx * my * mz) return false;
    px = k + t % mx;
    const int rest = t / mx;
    py = k + rest % my;
    pz = k + rest / my;
    return true;
}

template <typename real, int NX, int NY>
__device__ __forceinline__ real stencil_lds(const real *buf, int px, int py, int pz, real c0, real c1, real c2,
                                            real c3)
{
    constexpr int SY = NX, SZ = NX * NY;
    const real *p = buf + pz * SZ + py * SY + px;
    auto row = [&](int off, real &ctr, real &side) {
        ctr = p[off];
        side = p[off - 1] + p[off + 1];
    };
    real a, s, s0, s1, s2, s3;
    row(0, a, s);
    s0 = a;
    s1 = s;
    s2 = 0;
    s3 = 0;
    row(-SY, a, s); s1 += a; s2 += s;
    row(SY, a, s); s1 += a; s2 += s;
    row(-SZ, a, s); s1 += a; s2 += s;
    row(SZ, a, s); s1 += a; s2 += s;
    row(-SY - SZ, a, s); s2 += a; s3 += s;
    row(-SY + SZ, a, s); s2 += a; s3 += s;
    row(SY - SZ, a, s); s2 += a; s3 += s;
    row(SY + SZ, a, s); s2 += a; s3 += s;
    return c0 * s0 + c1 * s1 + c2 * s2 + c3 * s3;
}

// Decode the tile of this block from the tile plan.
template <int CX, int CY, int CZ>
__device__ __forceinline__ bool tile_of(const int *blk_rep, const int *blk_first, const Rep *rep, int &r, int &x0,
                                        int &y0, int &z0)
{
    r = blk_rep[plan_block()];
    const Rep &R = rep[r];
    const int ntx = (R.Lx + CX - 1) / CX, nty = (R.Ly + CY - 1) / CY;
    int lb = plan_block() - blk_first[r];
    x0 = (lb % ntx) * CX;
    lb /= ntx;
    y0 = (lb % nty) * CY;
    z0 = (lb / nty) * CZ;
    return true;
}

// Per-axis site offsets of the region positions (global index = ox[px] + oy[py] + oz[pz]).
template <int NX, int NY, int NZ>
__device__ __forceinline__ void region_offsets(const Rep &R, int x0, int y0, int z0, int K, int *ox, int *oy,
                                               int *oz)
{
    for (int t = threadIdx.x; t < NX + NY + NZ; t += kBlock) {
        if (t < NX) ox[t] = wrapn(x0 - K + t, R.Lx);
        else if (t < NX + NY) oy[t - NX] = wrapn(y0 - K + (t - NX), R.Ly) * R.Lx;
        else oz[t - NX - NY] = wrapn(z0 - K + (t - NX - NY), R.Lz) * R.Lx * R.Ly;
    }
}

// Forward sweep, steps s0+1 .. s0+nsteps (nsteps <= K).  G_{s0} is read from the
// store (G_0 = 1 when s0 = 0).  Partial sums per block (when `sums` is set, for the
// scale update): stored G_s over the core (rows s-1 of partG) and, when s0 = 0, E_A and
// E_B over the core (rows N, N+1); the row of G_N (for Q) is always written.
template <typename real, int CX, int CY, int CZ, int K>
__global__ __launch_bounds__(kBlock) void k_fwd_block(const int *__restrict__ blk_rep,
                                                      const int *__restrict__ blk_first,
                                                      const Rep *__restrict__ rep,
                                                      const RepState *__restrict__ st, Chain ch, int s0,
                                                      int nsteps, PropBufs<real> b, double *__restrict__ partG,
                                                      int nblocks, int sums)
{
    constexpr int NX = CX + 2 * K, NY = CY + 2 * K, NZ = CZ + 2 * K, NR = NX * NY * NZ;
    __shared__ real buf[2][NR];
    __shared__ int ox[NX], oy[NY], oz[NZ];
    int r, x0, y0, z0;
    tile_of<CX, CY, CZ>(blk_rep, blk_first, rep, r, x0, y0, z0);
    if (!st[r].active) return;
    const Rep &R = rep[r];
    const int V = (int)R.V;
    region_offsets<NX, NY, NZ>(R, x0, y0, z0, K, ox, oy, oz);
    const real c0 = (real)R.c[0], c1 = (real)R.c[1], c2 = (real)R.c[2], c3 = (real)R.c[3];
    real *G = b.G + (long long)ch.N * R.site_off;
    const real *E = b.E + off_poly(R);
    __syncthreads();
    // every global load of the launch is issued before the first is needed: the field
    // factors of all levels' sites of this thread, then G_{s0} on the full region
    constexpr int NIT = region_iters_total<CX, CY, CZ, K>();
    real ev[NIT];
    {
        int q = 0;
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            const real *Et = E + ch.types[min(s0 + k, ch.N) - 1] * V;
#pragma unroll
            for (int it = 0; it < region_iters<CX, CY, CZ, K>(k); ++it, ++q) {
                int px, py, pz;
                ev[q] = (real)0;
                if (k <= nsteps && region_pos<CX, CY, CZ, K>(k, it, px, py, pz)) ev[q] = Et[ox[px] + oy[py] + oz[pz]];
            }
        }
    }
    if (s0 == 0) {
        for (int t = threadIdx.x; t < NR; t += kBlock) buf[0][t] = (real)1;
    } else {
        const real *src = G + (long long)(s0 - 1) * V;
        for (int t = threadIdx.x; t < NR; t += kBlock) {
            const int px = t % NX, py = (t / NX) % NY, pz = t / (NX * NY);
            buf[0][t] = src[ox[px] + oy[py] + oz[pz]];
        }
    }
    __syncthreads();
    const int cx1 = min(CX, R.Lx - x0), cy1 = min(CY, R.Ly - y0), cz1 = min(CZ, R.Lz - z0);
    double esum[2] = {0.0, 0.0};
    int q = 0;
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        if (k > nsteps) break;
        const int s = s0 + k;
        const real sc = pow2_neg_b<real>(st[r].scale_e[s - 1]);
        const real *in = buf[(k - 1) & 1];
        real *out = buf[k & 1];
        double gsum = 0.0;
        q = 0;
#pragma unroll
        for (int kk = 1; kk < k; ++kk) q += region_iters<CX, CY, CZ, K>(kk);
#pragma unroll
        for (int it = 0; it < region_iters<CX, CY, CZ, K>(k); ++it) {
            int px, py, pz;
            if (!region_pos<CX, CY, CZ, K>(k, it, px, py, pz)) break;
            const int site = ox[px] + oy[py] + oz[pz];
            const real S = stencil_lds<real, NX, NY>(in, px, py, pz, c0, c1, c2, c3);
            const real g = ev[q + it] * S * sc;
            out[pz * NX * NY + py * NX + px] = g;
            const int qx = px - K, qy = py - K, qz = pz - K;
            if (qx >= 0 && qx < cx1 && qy >= 0 && qy < cy1 && qz >= 0 && qz < cz1) {
                G[(long long)(s - 1) * V + site] = g;
                gsum += (double)g;
                if (s == 1) {
                    esum[0] += (double)E[site];
                    esum[1] += (double)E[V + site];
                }
            }
        }
        if (sums || s == ch.N) {
            const double t = block_sum(gsum);   // contains __syncthreads: the level is complete
            if (threadIdx.x == 0) partG[(long long)(s - 1) * nblocks + plan_block()] = t;
        } else {
            __syncthreads();
        }
    }
    if (s0 == 0 && sums) {
        double t = block_sum(esum[0]);
        if (threadIdx.x == 0) partG[(long long)ch.N * nblocks + plan_block()] = t;
        t = block_sum(esum[1]);
        if (threadIdx.x == 0) partG[(long long)(ch.N + 1) * nblocks + plan_block()] = t;
    }
}

// Backward sweep, steps s_hi down to s_hi - nsteps + 1.  G+_{s_hi+1} is read from
// the ping-pong plane gin (G+_{N+1} = 1).  Accumulates G_s sigma[G+_{s+1}] per
// core site and species in LDS, then adds them to acc (or sets acc for the
// first launch).  The launch that reaches s = 1 normalises the densities:
// final_mode 0 writes phi (field layout), final_mode 1 writes g = phi^t - phi
// (polymer layout) with block partial sums d.g, g.z, |g_A|^2, |g_B|^2, where
// z = g / phi^t when the inversion is preconditioned and z = g otherwise.
template <typename real, int CX, int CY, int CZ, int K>
__global__ __launch_bounds__(kBlock) void k_bwd_block(const int *__restrict__ blk_rep,
                                                      const int *__restrict__ blk_first,
                                                      const Rep *__restrict__ rep,
                                                      const RepState *__restrict__ st, Chain ch, int s_hi,
                                                      int nsteps, PropBufs<real> b, const real *__restrict__ gin,
                                                      real *__restrict__ gout, double *__restrict__ acc,
                                                      int final_mode, const double *__restrict__ phit,
                                                      const double *__restrict__ d, double *__restrict__ out,
                                                      double *__restrict__ part)
{
    constexpr int NX = CX + 2 * K, NY = CY + 2 * K, NZ = CZ + 2 * K, NR = NX * NY * NZ;
    constexpr int NC = CX * CY * CZ;
    __shared__ real buf[2][NR];
    __shared__ double accl[2][NC];
    __shared__ int ox[NX], oy[NY], oz[NZ];
    int r, x0, y0, z0;
    tile_of<CX, CY, CZ>(blk_rep, blk_first, rep, r, x0, y0, z0);
    if (!st[r].active) return;
    const Rep &R = rep[r];
    const int V = (int)R.V;
    const int N = ch.N;
    region_offsets<NX, NY, NZ>(R, x0, y0, z0, K, ox, oy, oz);
    const real c0 = (real)R.c[0], c1 = (real)R.c[1], c2 = (real)R.c[2], c3 = (real)R.c[3];
    const real *G = b.G + (long long)N * R.site_off;
    const real *E = b.E + off_poly(R);
    for (int t = threadIdx.x; t < 2 * NC; t += kBlock) (&accl[0][0])[t] = 0.0;
    __syncthreads();
    // global loads issued up front: per level and site of this thread the field factor
    // (levels with s > 1) and, at core sites, G_s; then G+_{s_hi+1} on the region
    constexpr int NIT = region_iters_total<CX, CY, CZ, K>();
    real ev[NIT], gv[NIT];
    {
        int q = 0;
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            const int s = max(s_hi - k + 1, 1);
            const real *Et = E + ch.types[s - 1] * V;
            const real *Gs = G + (long long)(s - 1) * V;
#pragma unroll
            for (int it = 0; it < region_iters<CX, CY, CZ, K>(k); ++it, ++q) {
                int px, py, pz;
                ev[q] = gv[q] = (real)0;
                if (k <= nsteps && region_pos<CX, CY, CZ, K>(k, it, px, py, pz)) {
                    const int site = ox[px] + oy[py] + oz[pz];
                    if (s > 1) ev[q] = Et[site];
                    const int qx = px - K, qy = py - K, qz = pz - K;
                    if (qx >= 0 && qx < CX && qy >= 0 && qy < CY && qz >= 0 && qz < CZ) gv[q] = Gs[site];
                }
            }
        }
    }
    if (s_hi == N) {
        for (int t = threadIdx.x; t < NR; t += kBlock) buf[0][t] = (real)1;
    } else {
        const real *src = gin + R.site_off;
        for (int t = threadIdx.x; t < NR; t += kBlock) {
            const int px = t % NX, py = (t / NX) % NY, pz = t / (NX * NY);
            buf[0][t] = src[ox[px] + oy[py] + oz[pz]];
        }
    }
    __syncthreads();
    const int cx1 = min(CX, R.Lx - x0), cy1 = min(CY, R.Ly - y0), cz1 = min(CZ, R.Lz - z0);
    int last_k = 0;
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        if (k > nsteps) break;
        last_k = k;
        const int s = s_hi - k + 1;
        const int ts = ch.types[s - 1];
        const real sc = pow2_neg_b<real>(st[r].scale_e[s - 1]);
        const real *in = buf[(k - 1) & 1];
        real *o = buf[k & 1];
        int q = 0;
#pragma unroll
        for (int kk = 1; kk < k; ++kk) q += region_iters<CX, CY, CZ, K>(kk);
#pragma unroll
        for (int it = 0; it < region_iters<CX, CY, CZ, K>(k); ++it) {
            int px, py, pz;
            if (!region_pos<CX, CY, CZ, K>(k, it, px, py, pz)) break;
            const real S = stencil_lds<real, NX, NY>(in, px, py, pz, c0, c1, c2, c3);
            if (s > 1) o[pz * NX * NY + py * NX + px] = ev[q + it] * S * sc;
            const int qx = px - K, qy = py - K, qz = pz - K;
            if (qx >= 0 && qx < CX && qy >= 0 && qy < CY && qz >= 0 && qz < CZ)
                accl[ts][(qz * CY + qy) * CX + qx] += (double)gv[q + it] * (double)S;
        }
        __syncthreads();
    }
    const int s_lo = s_hi - last_k + 1;
    // core outputs: G+_{s_lo} for the next launch, accumulators, final densities
    const real *fin = buf[last_k & 1];
    const long long fo = off_field(R, ch.nsp), po = off_poly(R);
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    const double coef = st[r].phibar_p / ((double)N * st[r].q);
    for (int t = threadIdx.x; t < NC; t += kBlock) {
        const int qx = t % CX, qy = (t / CX) % CY, qz = t / (CX * CY);
        if (qx >= cx1 || qy >= cy1 || qz >= cz1) continue;
        const int px = qx + K, py = qy + K, pz = qz + K;
        const int site = ox[px] + oy[py] + oz[pz];
        if (s_lo > 1) gout[R.site_off + site] = fin[pz * NX * NY + py * NX + px];
        double a[2] = {accl[0][t], accl[1][t]};
        if (s_hi != N) {
            a[0] += acc[po + site];
            a[1] += acc[po + V + site];
        }
        if (s_lo > 1) {
            acc[po + site] = a[0];
            acc[po + V + site] = a[1];
        } else {
#pragma unroll
            for (int I = 0; I < 2; ++I) {
                const double ph = coef * a[I];
                if (final_mode == 0) {
                    out[fo + (long long)I * V + site] = ph;
                } else {
                    const double gI = phit[fo + (long long)I * V + site] - ph;
                    out[po + (long long)I * V + site] = gI;
                    if (d) sums[0] += d[po + (long long)I * V + site] * gI;
                    sums[1] += ch.precond ? gI * gI / phit[fo + (long long)I * V + site] : gI * gI;
                    sums[2 + I] += gI * gI;
                }
            }
        }
    }
    if (s_lo == 1 && final_mode == 1) {
        block_sums(sums);
        if (threadIdx.x == 0)
            for (int q = 0; q < 4; ++q) part[(long long)plan_block() * kNQ + q] = sums[q];
    }
}

// Replica of plan block pb and its descriptor, from a batch in the kernel arguments
// (constant indices only, so the descriptor stays in scalar registers).
__device__ __forceinline__ int arg_replica(const ArgReps &a, int pb)
{
    int r = 0;
#pragma unroll
    for (int k = 1; k < kArgReps; ++k)
        if (k < a.n && pb >= a.blk_first[k]) r = k;
    return r;
}

// The active flag of replica r as a vector load: its wait then joins the data loads of
// the step (a scalar load's result is waited for as soon as it is tested, which would put
// a round trip to memory before the first data load).
__device__ __forceinline__ int active_vec(const RepState *st, int r)
{
    return __hip_atomic_load(const_cast<int *>(&st[r].active), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ Rep arg_rep(const ArgReps &a, int r)
{
    static_assert(kArgReps == 4, "arg_rep selects among four replicas");
    return r == 0 ? a.rep[0] : (r == 1 ? a.rep[1] : (r == 2 ? a.rep[2] : a.rep[3]));
}

// E = exp(-(w + alpha d)) of the polymer species, all sites of the active replicas.
// ARGS: the batch is in the kernel arguments; the replica's active flag is then read
// alongside the fields and checked before the store.
template <typename real, bool ARGS>
__global__ __launch_bounds__(kBlock) void k_field_exp(const int *__restrict__ blk_rep,
                                                      const int *__restrict__ blk_first,
                                                      const Rep *__restrict__ rep,
                                                      const RepState *__restrict__ st, Chain ch,
                                                      const double *__restrict__ w, const double *__restrict__ d,
                                                      int use_alpha, real *__restrict__ E, ArgReps ar)
{
    int r;
    long long i;
    Rep R;
    int act = 1;   // read without a branch, tested before the store
    if (ARGS) {
        const int pb = plan_block();
        r = arg_replica(ar, pb);
        R = arg_rep(ar, r);
        i = (long long)(pb - ar.blk_first[r]) * kBlock + threadIdx.x;
        act = active_vec(st, r) | (ar.n == 1);
    } else {
        const SiteRef sr = site_ref(blk_rep, blk_first);
        r = sr.r;
        i = sr.i;
        if (!st[r].active) return;
        R = rep[r];
    }
    const long long V = R.V;
    if (i >= V) return;
    const long long fo = off_field(R, ch.nsp), po = off_poly(R);
    double x[2], dv[2] = {0.0, 0.0};
#pragma unroll
    for (int I = 0; I < 2; ++I) {
        x[I] = w[fo + I * V + i];
        if (use_alpha) dv[I] = d[po + I * V + i];
    }
    const double alpha = use_alpha ? st[r].alpha : 0.0;
    if (!act) return;
#pragma unroll
    for (int I = 0; I < 2; ++I) {
        if (use_alpha) x[I] = fma(alpha, dv[I], x[I]);
        E[po + I * V + i] = (real)exp(-x[I]);
    }
}

// One contour step per launch without LDS staging: the neighbours come through the
// caches.  Block tile CX x CY sites of a plane (CX * CY = kBlock threads, one (x, y)
// column each) and CZ consecutive planes per thread.  With CZ > 1 a thread forms, for
// every plane it touches, the in-plane class sums (centre, 4 edge-sharing, 4 corner
// neighbours: 9 loads) once and combines three consecutive planes per site, so a site
// costs 9 (CZ + 2) / CZ loads instead of 27.
// Tile of work item pb (a block's plan_block()) for the direct kernels and whether its
// replica is active.  ARGS:
// the batch is in the kernel arguments, so the stencil's loads need no dependent load
// before them; a one-replica context is active whenever a kernel is launched, the flag
// of a larger batch is loaded alongside the data and checked before the first store
// (the caller returns then, uniformly for the block).  Otherwise the tile plan and the
// descriptors come from device memory and an inactive replica returns at once.
template <int CX, int CY, int CZ, bool ARGS>
__device__ __forceinline__ void direct_tile(int pb, const int *blk_rep, const int *blk_first, const Rep *rep,
                                            const RepState *st, const ArgReps &ar, int &r, Rep &R, int &x0,
                                            int &y0, int &z0, int &act)
{
    int lb;
    if (ARGS) {
        r = arg_replica(ar, pb);
        R = arg_rep(ar, r);
        lb = pb - ar.blk_first[r];
        act = active_vec(st, r) | (ar.n == 1);   // no branch: the wait comes at the test
    } else {
        r = blk_rep[pb];
        R = rep[r];
        lb = pb - blk_first[r];
        act = st[r].active;
    }
    const int ntx = (R.Lx + CX - 1) / CX, nty = (R.Ly + CY - 1) / CY;
    x0 = (lb % ntx) * CX;
    lb /= ntx;
    y0 = (lb % nty) * CY;
    z0 = (lb / nty) * CZ;
}

// What a stencil applies to each loaded value before summing it: nothing, or (v m1) m2,
// the two products by which a backward step N forms G+_N = (E csum) sc from its field
// factor (so a stencil of the field factor through ScaleXf sums the values that step stores).
template <typename real>
struct NoXf {
    __device__ __forceinline__ real operator()(real v) const { return v; }
};
template <typename real>
struct ScaleXf {
    real m1, m2;
    __device__ __forceinline__ real operator()(real v) const { return (v * m1) * m2; }
};

// In-plane class sums of f around (x, y) in plane z (9 loads).
template <typename real, typename Xf = NoXf<real>>
__device__ __forceinline__ void plane_sums(const real *__restrict__ f, int x, int y, int z, int Lx, int Ly,
                                           real &a0, real &a1, real &a2, Xf xf = Xf())
{
    const int xm = wrap1(x - 1, Lx), xp = wrap1(x + 1, Lx);
    const int ym = wrap1(y - 1, Ly), yp = wrap1(y + 1, Ly);
    const real *p0 = f + ((long long)z * Ly + y) * Lx;
    const real *pm = f + ((long long)z * Ly + ym) * Lx;
    const real *pp = f + ((long long)z * Ly + yp) * Lx;
    a0 = xf(p0[x]);
    a1 = (xf(p0[xm]) + xf(p0[xp])) + (xf(pm[x]) + xf(pp[x]));
    a2 = (xf(pm[xm]) + xf(pm[xp])) + (xf(pp[xm]) + xf(pp[xp]));
}

// The same for tilings whose rows are 64 sites wide (a wavefront's lanes are consecutive x
// of one row): the x neighbours come from the adjacent lanes.  A lane whose neighbour lies
// outside the wavefront's row or across the box's periodic edge needs it from memory: with
// each row's centre every lane loads one more value, that outer neighbour if it is an edge
// lane and its own site otherwise, so the edge values arrive in the same round trip (a
// lane lacking both neighbours, in rows of one site, loads the right one after).  6 loads
// per plane instead of 9; same values summed in the same order as plane_sums.
template <typename real, typename Xf = NoXf<real>>
__device__ __forceinline__ void plane_sums_x64(const real *__restrict__ f, int x, int y, int z, int Lx, int Ly,
                                               real &a0, real &a1, real &a2, Xf xf = Xf())
{
    const int lane = (int)threadIdx.x & 63;
    const int ym = wrap1(y - 1, Ly), yp = wrap1(y + 1, Ly);
    const real *p0 = f + ((long long)z * Ly + y) * Lx;
    const real *pm = f + ((long long)z * Ly + ym) * Lx;
    const real *pp = f + ((long long)z * Ly + yp) * Lx;
    const bool lw = !(lane == 0 || x == 0), rw = !(lane == 63 || x == Lx - 1);
    const int xe = !lw ? wrap1(x - 1, Lx) : (!rw ? wrap1(x + 1, Lx) : x);
    const real c = xf(p0[x]), m = xf(pm[x]), p = xf(pp[x]);
    const real ce = xf(p0[xe]), me = xf(pm[xe]), pe = xf(pp[xe]);
    const real fcl = from_left(c), fml = from_left(m), fpl = from_left(p);
    const real fcr = from_right(c), fmr = from_right(m), fpr = from_right(p);
    real cl = lw ? fcl : ce, ml = lw ? fml : me, pl = lw ? fpl : pe;
    real cr = rw ? fcr : ce, mr = rw ? fmr : me, pr = rw ? fpr : pe;
    if (!lw && !rw) {
        const int xp = wrap1(x + 1, Lx);
        cr = xf(p0[xp]);
        mr = xf(pm[xp]);
        pr = xf(pp[xp]);
    }
    a0 = c;
    a1 = (cl + cr) + (m + p);
    a2 = (ml + mr) + (pl + pr);
}

// The stencil at the sites (x, y, z0 + j), j < nz (<= CZ), of f into S[j].  X64: rows of
// 64 lanes (plane_sums_x64); every lane of a row must take part.
template <typename real, int CZ, bool X64 = false, typename Xf = NoXf<real>>
__device__ __forceinline__ void column_stencil(const real *__restrict__ f, int x, int y, int z0, int nz, const Rep &R,
                                               real *S, Xf xf = Xf())
{
    const real c0 = (real)R.c[0], c1 = (real)R.c[1], c2 = (real)R.c[2], c3 = (real)R.c[3];
    if (CZ == 1 && !X64 && std::is_same<Xf, NoXf<real>>::value) {
        S[0] = stencil27<real>(f, x, y, z0, R.Lx, R.Ly, R.Lz, c0, c1, c2, c3);
        return;
    }
    real a0[CZ + 2], a1[CZ + 2], a2[CZ + 2];
    // planes z0 - 1 .. z0 + nz.  Short columns (CZ <= 2, the latency-bound small boxes):
    // past a short last chunk the plane index is clamped rather than branched on, so the
    // loads of every plane are issued together and wait once (values past the chunk are
    // not used).  Longer columns load plane by plane: issuing all of them at once costs
    // registers, and the occupancy that large boxes need to hide memory latency.
#pragma unroll
    for (int q = 0; q < CZ + 2; ++q) {
        if (CZ <= 2) {
            const int zq = wrap1(min(z0 - 1 + q, z0 + nz), R.Lz);
            if (X64) plane_sums_x64<real>(f, x, y, zq, R.Lx, R.Ly, a0[q], a1[q], a2[q], xf);
            else plane_sums<real>(f, x, y, zq, R.Lx, R.Ly, a0[q], a1[q], a2[q], xf);
        } else {
            a0[q] = a1[q] = a2[q] = (real)0;
            // the plane index is the same for every lane of a row, so a row stays together
            if (q <= nz + 1) {
                if (X64) plane_sums_x64<real>(f, x, y, wrap1(z0 - 1 + q, R.Lz), R.Lx, R.Ly, a0[q], a1[q], a2[q], xf);
                else plane_sums<real>(f, x, y, wrap1(z0 - 1 + q, R.Lz), R.Lx, R.Ly, a0[q], a1[q], a2[q], xf);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < CZ; ++j)
        S[j] = c0 * a0[j + 1] + c1 * (a1[j + 1] + (a0[j] + a0[j + 2])) + c2 * (a2[j + 1] + (a1[j] + a1[j + 2])) +
               c3 * (a2[j] + a2[j + 2]);
}

// Scalars of one contour-step launch, first among the kernel arguments so that they
// arrive with the first argument loads (read from the chain description they would take
// loads at step-dependent offsets): the step s, the chain length N, the species of beads
// s and 1, and the number of species.
struct StepInfo {
    int s, N, ts, t1, nsp;
};

inline StepInfo step_info(const Chain &ch, int s)
{
    return StepInfo{s, ch.N, ch.types[s - 1], ch.types[0], ch.nsp};
}

// With w set, step 1 also computes the field factors E = exp(-(w + alpha d)) of both
// polymer species at its sites (the tiles cover every site once) and stores them for the
// later steps, in place of a separate launch.
template <typename real, int CX, int CY, int CZ, bool ARGS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(real) == 4 ? 8 : 1))) void k_fwd_direct(StepInfo si, const int *__restrict__ blk_rep,
                                                       const int *__restrict__ blk_first,
                                                       const Rep *__restrict__ rep,
                                                       const RepState *__restrict__ st,
                                                       PropBufs<real> b, double *__restrict__ partG, int nblocks,
                                                       int sums, const double *__restrict__ w,
                                                       const double *__restrict__ dvec, int use_alpha, ArgReps ar)
{
    static_assert(CX * CY == kBlock, "one column per thread");
    int r, x0, y0, z0;
    Rep R;
    int act;
    direct_tile<CX, CY, CZ, ARGS>(plan_block(), blk_rep, blk_first, rep, st, ar, r, R, x0, y0, z0, act);
    if (!ARGS && !act) return;
    const int s = si.s;
    const int V = (int)R.V;
    const int x = x0 + (int)threadIdx.x % CX, y = y0 + (int)threadIdx.x / CX;
    const int nz = min(CZ, R.Lz - z0);
    const bool in = x < R.Lx && y < R.Ly;
    real *G = b.G + (long long)si.N * R.site_off;
    real *E = b.E + off_poly(R);
    const real *Es = E + si.ts * V;
    const bool fuse_exp = s == 1 && w != nullptr;
    // all loads of the step before the active check and the stores
    real S[CZ], Ev[CZ];
#pragma unroll
    for (int j = 0; j < CZ; ++j) S[j] = Ev[j] = (real)0;
    if (in) {
        if (s == 1) {
#pragma unroll
            for (int j = 0; j < CZ; ++j) S[j] = (real)R.csum;
        } else {
            column_stencil<real, CZ, CX == 64>(G + (long long)(s - 2) * V, x, y, z0, nz, R, S);
        }
        if (CZ <= 2 && !fuse_exp) {   // short columns: the field factors join the stencil's loads
#pragma unroll
            for (int j = 0; j < CZ; ++j) Ev[j] = Es[x + R.Lx * (y + R.Ly * min(z0 + j, z0 + nz - 1))];
        }
    }
    const real sc = pow2_neg_b<real>(st[r].scale_e[s - 1]);
    const double alpha = (fuse_exp && use_alpha) ? st[r].alpha : 0.0;
    if (!act) return;   // uniform for the block
    if (fuse_exp && in) {
        const long long fo = off_field(R, si.nsp), po = off_poly(R);
        const int t1 = si.t1;
#pragma unroll
        for (int j = 0; j < CZ; ++j) {
            if (j >= nz) break;
            const int site = x + R.Lx * (y + R.Ly * (z0 + j));
#pragma unroll
            for (int I = 0; I < 2; ++I) {
                double xv = w[fo + (long long)I * V + site];
                if (use_alpha) xv = fma(alpha, dvec[po + (long long)I * V + site], xv);
                const real e = (real)exp(-xv);
                E[(long long)I * V + site] = e;
                if (I == t1) Ev[j] = e;
            }
        }
    }
    double gsum = 0.0, esum[2] = {0.0, 0.0};
    if (in) {
#pragma unroll
        for (int j = 0; j < CZ; ++j) {
            if (j >= nz) break;
            const int site = x + R.Lx * (y + R.Ly * (z0 + j));
            const real g = ((CZ <= 2 || fuse_exp) ? Ev[j] : Es[site]) * S[j] * sc;
            G[(long long)(s - 1) * V + site] = g;
            gsum += (double)g;
            if (s == 1 && sums) {
                esum[0] += (double)E[site];
                esum[1] += (double)E[V + site];
            }
        }
    }
    if (sums || s == si.N) {
        const double t = block_sum(gsum);
        if (threadIdx.x == 0) partG[(long long)(s - 1) * nblocks + plan_block()] = t;
    }
    if (s == 1 && sums) {
        double t = block_sum(esum[0]);
        if (threadIdx.x == 0) partG[(long long)si.N * nblocks + plan_block()] = t;
        t = block_sum(esum[1]);
        if (threadIdx.x == 0) partG[(long long)(si.N + 1) * nblocks + plan_block()] = t;
    }
}

// FINAL: the launch of step 1 (only), which sums the stored density terms and normalises;
// the other steps' instances carry none of its registers.
// With fold_q = 1, step N's launch also finishes the forward sweep's reduction: the
// first block of each replica sums the replica's G_N partials (partG row N - 1, fixed
// order) and stores Q, ln Q and the range flag, which step 1 uses for the normalisation,
// in place of a separate control launch.  With fold_q = 2 (the paired sweeps, whose
// forward step N runs just before step 1), step 1's launch does it: every block sums the
// partials itself in that same order, so all hold the same Q, and the replica's first
// block stores it.
template <typename real, int CX, int CY, int CZ, bool ARGS, bool FINAL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(real) == 4 ? 8 : 1))) void k_bwd_direct(StepInfo si, const int *__restrict__ blk_rep,
                                                       const int *__restrict__ blk_first,
                                                       const Rep *__restrict__ rep,
                                                       RepState *__restrict__ st, Chain ch,
                                                       PropBufs<real> b, const real *__restrict__ gin,
                                                       real *__restrict__ gout, double *__restrict__ acc,
                                                       int final_mode, const double *__restrict__ phit,
                                                       const double *__restrict__ d, double *__restrict__ out,
                                                       double *__restrict__ part, const double *__restrict__ partG,
                                                       int nblocks, int fold_q, ArgReps ar)
{
    static_assert(CX * CY == kBlock, "one column per thread");
    int r, x0, y0, z0;
    Rep R;
    int act;
    direct_tile<CX, CY, CZ, ARGS>(plan_block(), blk_rep, blk_first, rep, st, ar, r, R, x0, y0, z0, act);
    if (!ARGS && !act) return;
    const int s = si.s;
    const int V = (int)R.V;
    const int N = si.N;
    const int ts = si.ts;
    const int x = x0 + (int)threadIdx.x % CX, y = y0 + (int)threadIdx.x / CX;
    const int nz = min(CZ, R.Lz - z0);
    const bool in = x < R.Lx && y < R.Ly;
    const long long po = off_poly(R);
    real *G = b.G + (long long)N * R.site_off;
    // the step's loads (stencil, field factor, stored G_s) before the active check
    real S[CZ], Ev[CZ], Gv[CZ];
#pragma unroll
    for (int j = 0; j < CZ; ++j) S[j] = Ev[j] = Gv[j] = (real)0;
    if (in) {
        if (s == N) {
#pragma unroll
            for (int j = 0; j < CZ; ++j) S[j] = (real)R.csum;
        } else {
            column_stencil<real, CZ, CX == 64>(gin + R.site_off, x, y, z0, nz, R, S);
        }
        if (CZ <= 2 && !FINAL) {   // short columns: all the step's loads go out together
#pragma unroll
            for (int j = 0; j < CZ; ++j) {
                // clamped past a short last chunk (those values are not used)
                const int site = x + R.Lx * (y + R.Ly * min(z0 + j, z0 + nz - 1));
                Ev[j] = b.E[po + ts * V + site];
                Gv[j] = G[(long long)(s - 1) * V + site];
            }
        }
    }
    // step 1 sums the stored terms of steps N .. 2 (slots N - 1 .. 1) in that order, then
    // its own: the first TB of them per plane, G_1 and (short columns, gradient mode) the
    // targets and the direction are loaded here with the stencil, for all planes together
    constexpr int TB = CZ <= 2 ? (sizeof(real) == 4 ? 32 : 16) / CZ : (sizeof(real) == 4 ? 2 : 1);
    real tv[CZ][TB], g1[CZ];
    double pt[CZ][2], pd[CZ][2];
#pragma unroll
    for (int j = 0; j < CZ; ++j) {
        g1[j] = (real)0;
        pt[j][0] = pt[j][1] = pd[j][0] = pd[j][1] = 0.0;
#pragma unroll
        for (int u = 0; u < TB; ++u) tv[j][u] = (real)0;
    }
    const long long fo = off_field(R, si.nsp);
    if (FINAL && in) {
#pragma unroll
        for (int j = 0; j < CZ; ++j) {
            const int site = x + R.Lx * (y + R.Ly * min(z0 + j, z0 + nz - 1));
            if (N >= 2) {
#pragma unroll
                for (int u = 0; u < TB; ++u) tv[j][u] = G[(long long)(max(N - u, 2) - 1) * V + site];
            }
            g1[j] = G[site];
            if (CZ <= 2 && final_mode == 1) {
#pragma unroll
                for (int I = 0; I < 2; ++I) {
                    pt[j][I] = phit[fo + (long long)I * V + site];
                    if (d) pd[j][I] = d[po + (long long)I * V + site];
                }
            }
        }
    }
    const real sc = pow2_neg_b<real>(st[r].scale_e[s - 1]);
    if (!act) return;   // uniform for the block
    if (fold_q == 1 && s == N && threadIdx.x < 64) {
        const int pb = plan_block();
        const int b0 = ARGS ? ar.blk_first[r] : blk_first[r], b1 = ARGS ? ar.blk_first[r + 1] : blk_first[r + 1];
        if (pb == b0) {
            double v = 0.0;
            const double *row = partG + (long long)(N - 1) * nblocks;
#pragma unroll 8
            for (int q = b0 + (int)threadIdx.x; q < b1; q += 64) v += row[q];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
            if (threadIdx.x == 0) {
                double q, lq;
                bool bad;
                q_from_sum(v, (double)R.V, st[r].scale_e, N, q, lq, bad);
                st[r].q = q;
                st[r].ln_q = lq;
                if (bad) st[r].nonfinite = 1;
            }
        }
    }
    // step 1: the sums of the stored terms per species (before the Q fold, whose partials
    // then take one more round trip)
    double a0[CZ], a1[CZ];
#pragma unroll
    for (int j = 0; j < CZ; ++j) a0[j] = a1[j] = 0.0;
    if (FINAL && in) {
        for (int q0 = N; q0 >= 2; q0 -= TB) {
            if (q0 != N) {
#pragma unroll
                for (int j = 0; j < CZ; ++j) {
                    const int site = x + R.Lx * (y + R.Ly * min(z0 + j, z0 + nz - 1));
#pragma unroll
                    for (int u = 0; u < TB; ++u) tv[j][u] = G[(long long)(max(q0 - u, 2) - 1) * V + site];
                }
            }
#pragma unroll
            for (int j = 0; j < CZ; ++j) {
#pragma unroll
                for (int u = 0; u < TB; ++u) {
                    const int q = q0 - u;
                    if (q < 2) break;
                    if (ch.types[q - 1] == 0) a0[j] += (double)tv[j][u];
                    else a1[j] += (double)tv[j][u];
                }
            }
        }
    }
    double q_own = 0.0;
    if (FINAL && fold_q == 2) {
        __shared__ double q_sh;
        if (threadIdx.x < 64) {
            const int pb = plan_block();
            const int b0 = ARGS ? ar.blk_first[r] : blk_first[r], b1 = ARGS ? ar.blk_first[r + 1] : blk_first[r + 1];
            double v = 0.0;
            const double *row = partG + (long long)(N - 1) * nblocks;
#pragma unroll 8
            for (int q = b0 + (int)threadIdx.x; q < b1; q += 64) v += row[q];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
            if (threadIdx.x == 0) {
                double q, lq;
                bool bad;
                q_from_sum(v, (double)R.V, st[r].scale_e, N, q, lq, bad);
                q_sh = q;
                if (pb == b0) {
                    st[r].q = q;
                    st[r].ln_q = lq;
                    if (bad) st[r].nonfinite = 1;
                }
            }
        }
        __syncthreads();
        q_own = q_sh;
    }
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    if (in && !FINAL) {
#pragma unroll
        for (int j = 0; j < CZ; ++j) {
            if (j >= nz) break;
            const int site = x + R.Lx * (y + R.Ly * (z0 + j));
            real *Gs = G + (long long)(s - 1) * V + site;
            const real e = CZ <= 2 ? Ev[j] : b.E[po + ts * V + site];
            const real gs = CZ <= 2 ? Gv[j] : *Gs;
            gout[R.site_off + site] = e * S[j] * sc;
            // the density term G_s sigma[G+_{s+1}] replaces G_s in the store (G_s is
            // not read again in this evaluation); step 1 sums them
            *Gs = gs * S[j];
        }
    }
    if (in && FINAL) {
        const double coef = st[r].phibar_p / ((double)N * (fold_q == 2 ? q_own : st[r].q));
#pragma unroll
        for (int j = 0; j < CZ; ++j) {
            if (j >= nz) break;
            const int site = x + R.Lx * (y + R.Ly * (z0 + j));
            double a[2] = {a0[j], a1[j]};
            a[ts] += (double)g1[j] * (double)S[j];
#pragma unroll
            for (int I = 0; I < 2; ++I) {
                const double ph = coef * a[I];
                if (final_mode == 0) {
                    out[fo + (long long)I * V + site] = ph;
                } else {
                    const double tI = CZ <= 2 ? pt[j][I] : phit[fo + (long long)I * V + site];
                    const double gI = tI - ph;
                    out[po + (long long)I * V + site] = gI;
                    if (d) sums[0] += (CZ <= 2 ? pd[j][I] : d[po + (long long)I * V + site]) * gI;
                    sums[1] += ch.precond ? gI * gI / tI : gI * gI;
                    sums[2 + I] += gI * gI;
                }
            }
        }
    }
    if (FINAL && final_mode == 1) {
        block_sums(sums);
        if (threadIdx.x == 0)
            for (int q = 0; q < 4; ++q) part[(long long)plan_block() * kNQ + q] = sums[q];
    }
}

// ---- paired sweeps ------------------------------------------------------------------
//
// The backward propagators G+_s do not depend on the forward ones (both start from the
// field factors), so one launch can advance the forward sweep by a step and the backward
// sweep by a step: its first pi.nf blocks take forward step pi.f.s, the rest backward step
// pi.g.s, with the same tiling.  A bead's density term G_s sigma[G+_{s+1}] is formed by
// whichever of its two steps runs second.  Early forward steps (s <= the crossing) store
// G_s in slot s - 1 as the one-step kernels do, and the backward step of that bead later
// replaces it by the term.  Early backward steps (s above the crossing) store
// sigma_s = sigma[G+_{s+1}] in slot s - 1, and the forward step of that bead later reads
// it and replaces it by the term; from the crossing on the forward propagator moves
// through its own ping-pong pair (fin -> fout), since its slots are taken.  Every stored
// value is the same expression of the same operands as in the one-step sequence, so the
// densities are bit for bit those of that sequence.  Step 1 of the backward sweep, which
// sums the terms, runs in a launch of its own after the last paired one.
struct PairInfo {
    StepInfo f, g;   // forward and backward step (s = 0: none)
    int f_late;      // forward: sigma_s is in slot s - 1 and the term replaces it
    int f_from_pp;   // forward: G_{s-1} is read from fin (else from slot s - 2)
    int f_to_pp;     // forward: G_s is also written to fout
    int g_late;      // backward: G_s is in slot s - 1 and the term replaces it (else sigma_s is stored)
    int g_exp;       // backward: the field factor is computed from w here (step 1's launch, same values)
    int g_from_e;    // backward step N - 1: its stencil reads G+_N as bead N's field factor times csum
                     // and the step-N scale, the two products backward step N would store
    int g_tn;        // species of bead N
    int nf;          // blocks of the forward half (0 or the tile plan's count)
};

template <typename real, int CX, int CY, int CZ, bool ARGS>
__device__ __forceinline__ void pair_fwd(const PairInfo &pi, int pb, const int *__restrict__ blk_rep,
                                         const int *__restrict__ blk_first, const Rep *__restrict__ rep,
                                         const RepState *__restrict__ st, PropBufs<real> b,
                                         const real *__restrict__ fin, real *__restrict__ fout,
                                         double *__restrict__ partG, int nblocks, int sums,
                                         const double *__restrict__ w, const double *__restrict__ dvec,
                                         int use_alpha, const ArgReps &ar)
{
    int r, x0, y0, z0;
    Rep R;
    int act;
    direct_tile<CX, CY, CZ, ARGS>(pb, blk_rep, blk_first, rep, st, ar, r, R, x0, y0, z0, act);
    if (!ARGS && !act) return;
    const StepInfo si = pi.f;
    const int s = si.s, N = si.N;
    const int V = (int)R.V;
    const int x = x0 + (int)threadIdx.x % CX, y = y0 + (int)threadIdx.x / CX;
    const int nz = min(CZ, R.Lz - z0);
    const bool in = x < R.Lx && y < R.Ly;
    real *G = b.G + (long long)N * R.site_off;
    real *E = b.E + off_poly(R);
    const real *Es = E + si.ts * V;
    const bool fuse_exp = s == 1 && w != nullptr;
    const bool late = pi.f_late != 0, sig_in = late && s < N;
    real S[CZ], Ev[CZ], Sg[CZ];
#pragma unroll
    for (int j = 0; j < CZ; ++j) S[j] = Ev[j] = Sg[j] = (real)0;
    if (in) {
        if (s == 1) {
#pragma unroll
            for (int j = 0; j < CZ; ++j) S[j] = (real)R.csum;
        } else {
            column_stencil<real, CZ, CX == 64>(pi.f_from_pp ? fin + R.site_off : G + (long long)(s - 2) * V, x, y, z0, nz, R, S);
        }
        if (CZ <= 2) {
#pragma unroll
            for (int j = 0; j < CZ; ++j) {
                const int site = x + R.Lx * (y + R.Ly * min(z0 + j, z0 + nz - 1));
                if (!fuse_exp) Ev[j] = Es[site];
                if (sig_in) Sg[j] = G[(long long)(s - 1) * V + site];
            }
        }
    }
    const real sc = pow2_neg_b<real>(st[r].scale_e[s - 1]);
    const double alpha = (fuse_exp && use_alpha) ? st[r].alpha : 0.0;
    if (!act) return;   // uniform for the block
    if (fuse_exp && in) {
        const long long fo = off_field(R, si.nsp), po = off_poly(R);
        const int t1 = si.t1;
#pragma unroll
        for (int j = 0; j < CZ; ++j) {
            if (j >= nz) break;
            const int site = x + R.Lx * (y + R.Ly * (z0 + j));
#pragma unroll
            for (int I = 0; I < 2; ++I) {
                double xv = w[fo + (long long)I * V + site];
                if (use_alpha) xv = fma(alpha, dvec[po + (long long)I * V + site], xv);
                const real e = (real)exp(-xv);
                E[(long long)I * V + site] = e;
                if (I == t1) Ev[j] = e;
            }
        }
    }
    double gsum = 0.0, esum[2] = {0.0, 0.0};
    if (in) {
#pragma unroll
        for (int j = 0; j < CZ; ++j) {
            if (j >= nz) break;
            const int site = x + R.Lx * (y + R.Ly * (z0 + j));
            const real g = ((CZ <= 2 || fuse_exp) ? Ev[j] : Es[site]) * S[j] * sc;
            real *slot = G + (long long)(s - 1) * V + site;
            if (late) {
                const real sg = s == N ? (real)R.csum : (CZ <= 2 ? Sg[j] : *slot);
                *slot = g * sg;
            } else {
                *slot = g;
            }
            if (pi.f_to_pp) fout[R.site_off + site] = g;
            gsum += (double)g;
            if (s == 1 && sums) {
                esum[0] += (double)E[site];
                esum[1] += (double)E[V + site];
            }
        }
    }
    if (sums || s == N) {
        const double t = block_sum(gsum);
        if (threadIdx.x == 0) partG[(long long)(s - 1) * nblocks + pb] = t;
    }
    if (s == 1 && sums) {
        double t = block_sum(esum[0]);
        if (threadIdx.x == 0) partG[(long long)N * nblocks + pb] = t;
        t = block_sum(esum[1]);
        if (threadIdx.x == 0) partG[(long long)(N + 1) * nblocks + pb] = t;
    }
}

template <typename real, int CX, int CY, int CZ, bool ARGS>
__device__ __forceinline__ void pair_bwd(const PairInfo &pi, int pb, const int *__restrict__ blk_rep,
                                         const int *__restrict__ blk_first, const Rep *__restrict__ rep,
                                         const RepState *__restrict__ st, PropBufs<real> b,
                                         const real *__restrict__ gin, real *__restrict__ gout,
                                         const double *__restrict__ w, const double *__restrict__ dvec,
                                         int use_alpha, const ArgReps &ar)
{
    int r, x0, y0, z0;
    Rep R;
    int act;
    direct_tile<CX, CY, CZ, ARGS>(pb, blk_rep, blk_first, rep, st, ar, r, R, x0, y0, z0, act);
    if (!ARGS && !act) return;
    const StepInfo si = pi.g;
    const int s = si.s, N = si.N, ts = si.ts;
    const int V = (int)R.V;
    const int x = x0 + (int)threadIdx.x % CX, y = y0 + (int)threadIdx.x / CX;
    const int nz = min(CZ, R.Lz - z0);
    const bool in = x < R.Lx && y < R.Ly;
    const long long po = off_poly(R);
    real *G = b.G + (long long)N * R.site_off;
    const bool late = pi.g_late != 0, fexp = pi.g_exp != 0;
    real S[CZ], Ev[CZ], Gv[CZ];
#pragma unroll
    for (int j = 0; j < CZ; ++j) S[j] = Ev[j] = Gv[j] = (real)0;
    if (in) {
        if (s == N) {
#pragma unroll
            for (int j = 0; j < CZ; ++j) S[j] = (real)R.csum;
        } else if (pi.g_from_e) {
            const ScaleXf<real> xf{(real)R.csum, pow2_neg_b<real>(st[r].scale_e[N - 1])};
            column_stencil<real, CZ, CX == 64>(b.E + po + (long long)pi.g_tn * V, x, y, z0, nz, R, S, xf);
        } else {
            column_stencil<real, CZ, CX == 64>(gin + R.site_off, x, y, z0, nz, R, S);
        }
        if (CZ <= 2) {
#pragma unroll
            for (int j = 0; j < CZ; ++j) {
                const int site = x + R.Lx * (y + R.Ly * min(z0 + j, z0 + nz - 1));
                if (!fexp) Ev[j] = b.E[po + ts * V + site];
                if (late) Gv[j] = G[(long long)(s - 1) * V + site];
            }
        }
    }
    const real sc = pow2_neg_b<real>(st[r].scale_e[s - 1]);
    const double alpha = (fexp && use_alpha) ? st[r].alpha : 0.0;
    if (!act) return;   // uniform for the block
    if (in) {
        const long long fo = off_field(R, si.nsp);
#pragma unroll
        for (int j = 0; j < CZ; ++j) {
            if (j >= nz) break;
            const int site = x + R.Lx * (y + R.Ly * (z0 + j));
            real e;
            if (fexp) {
                double xv = w[fo + (long long)ts * V + site];
                if (use_alpha) xv = fma(alpha, dvec[po + (long long)ts * V + site], xv);
                e = (real)exp(-xv);
            } else {
                e = CZ <= 2 ? Ev[j] : b.E[po + ts * V + site];
            }
            gout[R.site_off + site] = e * S[j] * sc;
            real *slot = G + (long long)(s - 1) * V + site;
            if (late) {
                const real gs = CZ <= 2 ? Gv[j] : *slot;
                *slot = gs * S[j];
            } else if (s < N) {
                *slot = S[j];
            }
        }
    }
}

template <typename real, int CX, int CY, int CZ, bool ARGS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(real) == 4 ? 8 : 1))) void k_pair_direct(PairInfo pi, const int *__restrict__ blk_rep,
                                                        const int *__restrict__ blk_first,
                                                        const Rep *__restrict__ rep,
                                                        const RepState *__restrict__ st, PropBufs<real> b,
                                                        const real *__restrict__ fin, real *__restrict__ fout,
                                                        const real *__restrict__ gin, real *__restrict__ gout,
                                                        double *__restrict__ partG, int nblocks, int sums,
                                                        const double *__restrict__ w,
                                                        const double *__restrict__ dvec, int use_alpha, ArgReps ar)
{
    static_assert(CX * CY == kBlock, "one column per thread");
    const int pb = plan_block();
    if (pb < pi.nf)
        pair_fwd<real, CX, CY, CZ, ARGS>(pi, pb, blk_rep, blk_first, rep, st, b, fin, fout, partG, nblocks, sums, w,
                                         dvec, use_alpha, ar);
    else
        pair_bwd<real, CX, CY, CZ, ARGS>(pi, pb - pi.nf, blk_rep, blk_first, rep, st, b, gin, gout, w, dvec,
                                         use_alpha, ar);
}

// ---- launchers ---------------------------------------------------------------------

template <typename real, int CX, int CY, int CZ, int K>
struct BlockKernels {
    static void fwd(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, int s0, int n,
                    PropBufs<real> b, double *partG, int sums, const double *w, const double *d, int use_alpha,
                    hipEvent_t e0, hipEvent_t e1)
    {
        if constexpr (K <= 0) {   // direct kernels (K = -1: their single steps)
            auto kern = p.args.n ? k_fwd_direct<real, CX, CY, CZ, true> : k_fwd_direct<real, CX, CY, CZ, false>;
            if (e0)
                hipExtLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), 0, s, e0, e1, 0, step_info(ch, s0 + 1),
                                      p.blk_rep, p.blk_first, rep, st, b, partG, p.nblocks, sums, w, d, use_alpha,
                                      p.args);
            else
                hipLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), 0, s, step_info(ch, s0 + 1), p.blk_rep,
                                   p.blk_first, rep, st, b, partG, p.nblocks, sums, w, d, use_alpha, p.args);
        } else {
            if (e0)
                hipExtLaunchKernelGGL((k_fwd_block<real, CX, CY, CZ, K>), dim3(p.nblocks), dim3(kBlock), 0, s, e0,
                                      e1, 0, p.blk_rep, p.blk_first, rep, st, ch, s0, n, b, partG, p.nblocks, sums);
            else
                hipLaunchKernelGGL((k_fwd_block<real, CX, CY, CZ, K>), dim3(p.nblocks), dim3(kBlock), 0, s,
                                   p.blk_rep, p.blk_first, rep, st, ch, s0, n, b, partG, p.nblocks, sums);
        }
    }
    static void bwd(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, int s_hi, int n,
                    PropBufs<real> b, const real *gin, real *gout, double *acc, int final_mode, const double *phit,
                    const double *d, double *out, double *part, const double *partG, int fold_q, hipEvent_t e0,
                    hipEvent_t e1)
    {
        if constexpr (K <= 0) {   // direct kernels (K = -1: their single steps)
            auto kern = s_hi == 1 ? (p.args.n ? k_bwd_direct<real, CX, CY, CZ, true, true>
                                              : k_bwd_direct<real, CX, CY, CZ, false, true>)
                                  : (p.args.n ? k_bwd_direct<real, CX, CY, CZ, true, false>
                                              : k_bwd_direct<real, CX, CY, CZ, false, false>);
            if (e0)
                hipExtLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), 0, s, e0, e1, 0, step_info(ch, s_hi),
                                      p.blk_rep, p.blk_first, rep, st, ch, b, gin, gout, acc, final_mode, phit, d,
                                      out, part, partG, p.nblocks, fold_q, p.args);
            else
                hipLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), 0, s, step_info(ch, s_hi), p.blk_rep,
                                   p.blk_first, rep, st, ch, b, gin, gout, acc, final_mode, phit, d, out, part, partG,
                                   p.nblocks, fold_q, p.args);
        } else {
            if (e0)
                hipExtLaunchKernelGGL((k_bwd_block<real, CX, CY, CZ, K>), dim3(p.nblocks), dim3(kBlock), 0, s, e0,
                                      e1, 0, p.blk_rep, p.blk_first, rep, st, ch, s_hi, n, b, gin, gout, acc,
                                      final_mode, phit, d, out, part);
            else
                hipLaunchKernelGGL((k_bwd_block<real, CX, CY, CZ, K>), dim3(p.nblocks), dim3(kBlock), 0, s,
                                   p.blk_rep, p.blk_first, rep, st, ch, s_hi, n, b, gin, gout, acc, final_mode,
                                   phit, d, out, part);
        }
    }
};

// One paired launch (tiles of the K = -1 configurations): forward step sf and backward
// step sb (0: none).
template <typename real, int CX, int CY, int CZ>
void pair_launch(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, const PairSteps &ps,
                 PropBufs<real> b, const real *fin, real *fout, const real *gin, real *gout, double *partG,
                 int sums, const double *w, const double *d, int use_alpha, hipEvent_t e0, hipEvent_t e1)
{
    PairInfo pi{};
    if (ps.sf) pi.f = step_info(ch, ps.sf);
    if (ps.sb) pi.g = step_info(ch, ps.sb);
    pi.f_late = ps.f_late;
    pi.f_from_pp = ps.f_from_pp;
    pi.f_to_pp = ps.f_to_pp;
    pi.g_late = ps.g_late;
    pi.g_exp = ps.g_exp;
    pi.g_from_e = ps.g_from_e;
    pi.g_tn = ch.types[ch.N - 1];
    pi.nf = ps.sf ? p.nblocks : 0;
    const int grid = pi.nf + (ps.sb ? p.nblocks : 0);
    auto kern = p.args.n ? k_pair_direct<real, CX, CY, CZ, true> : k_pair_direct<real, CX, CY, CZ, false>;
    if (e0)
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, e0, e1, 0, pi, p.blk_rep, p.blk_first, rep, st, b,
                              fin, fout, gin, gout, partG, p.nblocks, sums, w, d, use_alpha, p.args);
    else
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, pi, p.blk_rep, p.blk_first, rep, st, b, fin, fout,
                           gin, gout, partG, p.nblocks, sums, w, d, use_alpha, p.args);
}

template <typename real>
void launch_pair_block(const TileCfg &cfg, hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                       const PairSteps &ps, PropBufs<real> b, const real *fin, real *fout, const real *gin,
                       real *gout, double *partG, int sums, const double *w, const double *d, int use_alpha,
                       hipEvent_t e0, hipEvent_t e1)
{
#define HSF_CASE(CX, CY, CZ, K)                                                                             \
    if constexpr (K == -1)                                                                                  \
        if (cfg.cx == CX && cfg.cy == CY && cfg.cz == CZ && cfg.k == K)                                     \
            return pair_launch<real, CX, CY, CZ>(s, p, rep, st, ch, ps, b, fin, fout, gin, gout, partG, sums, w, \
                                                 d, use_alpha, e0, e1);
    HSF_TILE_CONFIGS(HSF_CASE)
#undef HSF_CASE
}

template <typename real>
void launch_field_exp(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, const double *w,
                      const double *d, int use_alpha, real *E, hipEvent_t e0, hipEvent_t e1)
{
    auto kern = p.args.n ? k_field_exp<real, true> : k_field_exp<real, false>;
    if (e0)
        hipExtLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), 0, s, e0, e1, 0, p.blk_rep, p.blk_first, rep, st,
                              ch, w, d, use_alpha, E, p.args);
    else
        hipLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, st, ch, w, d,
                           use_alpha, E, p.args);
}

template <typename real>
void launch_fwd_block(const TileCfg &cfg, hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                      int s0, int n, PropBufs<real> b, double *partG, int sums, const double *w, const double *d,
                      int use_alpha, hipEvent_t e0, hipEvent_t e1)
{
#define HSF_CASE(CX, CY, CZ, K)                                                                   \
    if (cfg.cx == CX && cfg.cy == CY && cfg.cz == CZ && cfg.k == K)                               \
        return BlockKernels<real, CX, CY, CZ, K>::fwd(s, p, rep, st, ch, s0, n, b, partG, sums, w, d, use_alpha, \
                                                      e0, e1);
    HSF_TILE_CONFIGS(HSF_CASE)
#undef HSF_CASE
}

template <typename real>
void launch_bwd_block(const TileCfg &cfg, hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                      int s_hi, int n, PropBufs<real> b, const real *gin, real *gout, double *acc, int final_mode,
                      const double *phit, const double *d, double *out, double *part, const double *partG,
                      int fold_q, hipEvent_t e0, hipEvent_t e1)
{
#define HSF_CASE(CX, CY, CZ, K)                                                                        \
    if (cfg.cx == CX && cfg.cy == CY && cfg.cz == CZ && cfg.k == K)                                    \
        return BlockKernels<real, CX, CY, CZ, K>::bwd(s, p, rep, st, ch, s_hi, n, b, gin, gout, acc,       \
                                                      final_mode, phit, d, out, part, partG, fold_q, e0, e1);
    HSF_TILE_CONFIGS(HSF_CASE)
#undef HSF_CASE
}

#define HSF_INST(real)                                                                                    \
    template void launch_field_exp<real>(hipStream_t, const Plan &, const Rep *, RepState *, Chain,       \
                                         const double *, const double *, int, real *, hipEvent_t,         \
                                         hipEvent_t);                                                     \
    template void launch_fwd_block<real>(const TileCfg &, hipStream_t, const Plan &, const Rep *,         \
                                         RepState *, Chain, int, int, PropBufs<real>, double *, int,      \
                                         const double *, const double *, int, hipEvent_t, hipEvent_t);    \
    template void launch_bwd_block<real>(const TileCfg &, hipStream_t, const Plan &, const Rep *,         \
                                         RepState *, Chain, int, int, PropBufs<real>, const real *,       \
                                         real *, double *, int, const double *, const double *, double *, \
                                         double *, const double *, int, hipEvent_t, hipEvent_t);          \
    template void launch_pair_block<real>(const TileCfg &, hipStream_t, const Plan &, const Rep *,        \
                                          RepState *, Chain, const PairSteps &, PropBufs<real>,          \
                                          const real *, real *, const real *, real *, double *, int,     \
                                          const double *, const double *, int, hipEvent_t, hipEvent_t);
HSF_INST(double)
HSF_INST(float)
#undef HSF_INST

}  // namespace hsf
