// prop_stream.hip -- z-streaming, temporally blocked propagator sweeps (eq. 16-17).
//
// One launch advances K contour steps.  A wavefront owns a tile of the (x, y) plane and
// walks along z: its 64 lanes are 64 consecutive x sites (periodic), each lane holds H
// consecutive y rows in registers, and the K levels (contour steps) form a pipeline in z:
// when plane q of level l - 1 is known, its in-plane class sums (centre, 4 edge-sharing,
// 4 corner neighbours; x neighbours through lane shifts, y neighbours from the lane's own
// rows) complete plane q - 1 of level l and are pushed into the pending sums of planes
// q and q + 1.  Levels shrink by one site per side per step in x and y, so a tile's core
// is (64 - 2K) x (H - 2K) columns of a z-chunk, and its halo is recomputed by the
// neighbouring tiles; nothing goes through LDS.  Per launch the propagator is read once
// (level 0, with its halo) and written once per level at the core (forward store) or once
// at the last level (backward ping-pong), so a site-bead update moves about
// s_G (1 + 2 / K) bytes of propagator instead of 3 s_G for one step per launch.
//
// Backward launches accumulate the density terms G_s sigma[G+_{s+1}] of their levels per
// site and species and store the partial sums in the propagator-store slots they have
// just consumed (G_s is not read again); the launch that reaches s = 1 adds the partial
// sums of the earlier launches to its own and normalises (eq. 2, 16).  Scaling as in the
// other sweeps: the per-step powers of two divide both G_s and G+_s.
#include <hip/hip_ext.h>

#include "device_common.h"
#include "prop_block.h"

namespace hsf {

namespace {

__device__ __forceinline__ int wrapm(int v, int L)
{
    v %= L;
    return v < 0 ? v + L : v;
}

template <typename real>
__device__ __forceinline__ real pow2_neg(int e)
{
    return (real)ldexp(1.0, -e);
}

// Tile of wavefront `tile` (index within its replica) for core widths of at most
// WX = 64 - 2K columns and WY = H - 2K rows: the box is cut into ntx x nty x ntz tiles of
// near-equal cores (the host's plan counts the same tiles).
template <int K, int H>
struct STile {
    int x0, y0, z0;      // core origin
    int cx, cy, cz;      // core extent (ragged at the box's end)
    bool live;
};

template <int K, int H>
__device__ __forceinline__ STile<K, H> stream_tile(const Rep &R, int cz, int tile)
{
    constexpr int WX = 64 - 2 * K, WY = H - 2 * K;
    const int ntx = (R.Lx + WX - 1) / WX, nty = (R.Ly + WY - 1) / WY, ntz = (R.Lz + cz - 1) / cz;
    const int cx = (R.Lx + ntx - 1) / ntx, cy = (R.Ly + nty - 1) / nty;
    STile<K, H> t;
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    t.x0 = tx * cx;
    t.y0 = ty * cy;
    t.z0 = tz * cz;
    t.live = tz < ntz && t.x0 < R.Lx && t.y0 < R.Ly;
    t.cx = min(cx, R.Lx - t.x0);
    t.cy = min(cy, R.Ly - t.y0);
    t.cz = min(cz, R.Lz - t.z0);
    return t;
}

// Replica of plan block pb (kernel arguments for small batches, tables otherwise).
__device__ __forceinline__ int stream_replica(int pb, const int *blk_rep, const ArgReps &ar)
{
    if (ar.n) {
        int r = 0;
#pragma unroll
        for (int k = 1; k < kArgReps; ++k)
            if (k < ar.n && pb >= ar.blk_first[k]) r = k;
        return r;
    }
    return blk_rep[pb];
}

__device__ __forceinline__ Rep stream_rep(const ArgReps &ar, const Rep *rep, int r)
{
    static_assert(kArgReps == 4, "selects among four replicas");
    if (ar.n) return r == 0 ? ar.rep[0] : (r == 1 ? ar.rep[1] : (r == 2 ? ar.rep[2] : ar.rep[3]));
    return rep[r];
}

// One level of the pipeline on one plane: in-plane class sums of the level below (f),
// pushed into the pending sums (P: plane q, U: contribution u of plane q - 1 to q); returns
// the completed stencil of plane q - 1 in S.
template <typename real, int H>
__device__ __forceinline__ void stencil_push(const real (&f)[H], real (&P)[H], real (&U)[H], real (&S)[H], real c0,
                                             real c1, real c2, real c3)
{
    real h1[H];
#pragma unroll
    for (int j = 0; j < H; ++j) h1[j] = from_left(f[j]) + from_right(f[j]);
#pragma unroll
    for (int j = 0; j < H; ++j) {
        // rows 0 and H - 1 lack a neighbour: they are halo, never valid past level 0
        const real fm = j > 0 ? f[j - 1] : (real)0, fp = j < H - 1 ? f[j + 1] : (real)0;
        const real hm = j > 0 ? h1[j - 1] : (real)0, hp = j < H - 1 ? h1[j + 1] : (real)0;
        const real a0 = f[j], a1 = h1[j] + (fm + fp), a2 = hm + hp;
        const real u = c1 * a0 + c2 * a1 + c3 * a2;   // to the planes above and below
        const real v = c0 * a0 + c1 * a1 + c2 * a2;   // to its own plane
        S[j] = P[j] + u;
        P[j] = U[j] + v;
        U[j] = u;
    }
}

}  // namespace

// Forward sweep, steps s0 + 1 .. s0 + nsteps (nsteps <= K), from G_{s0} in the store
// (G_0 = 1).  Stores G_s at the core of every level; per-block sums of the stored G_s
// (rows s - 1 of partG, when `sums` or s = N) and, with s0 = 0 and `sums`, of E_A and E_B
// (rows N, N + 1).  Every load of plane iteration i + 1 is issued before iteration i
// computes, so a wavefront waits for memory once per plane.
template <typename real, int K, int H>
__global__ __launch_bounds__(kBlock) void k_fwd_stream(const int *__restrict__ blk_rep,
                                                       const int *__restrict__ blk_first,
                                                       const Rep *__restrict__ rep,
                                                       const RepState *__restrict__ st, Chain ch, int s0, int nsteps,
                                                       int cz, PropBufs<real> b, double *__restrict__ partG,
                                                       int nblocks, int sums, ArgReps ar)
{
    const int pb = plan_block();
    const int r = stream_replica(pb, blk_rep, ar);
    if (!st[r].active && ar.n != 1) return;   // uniform for the block
    const Rep R = stream_rep(ar, rep, r);
    const int bf = ar.n ? ar.blk_first[r] : blk_first[r];
    const int wv = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const STile<K, H> t = stream_tile<K, H>(R, cz, (pb - bf) * (kBlock / 64) + wv);
    const unsigned V = (unsigned)R.V, LxLy = (unsigned)(R.Lx * R.Ly);
    const real c0 = (real)R.c[0], c1 = (real)R.c[1], c2 = (real)R.c[2], c3 = (real)R.c[3];
    real *G = b.G + (long long)ch.N * R.site_off;
    const real *E = b.E + off_poly(R);
    const int x = wrapm(t.x0 - K + lane, R.Lx);
    const bool xcore = lane >= K && lane < K + t.cx;
    unsigned yo[H];
#pragma unroll
    for (int j = 0; j < H; ++j) yo[j] = (unsigned)(wrapm(t.y0 - K + j, R.Ly) * R.Lx + x);
    const real *Gin = s0 > 0 ? G + (size_t)(s0 - 1) * V : nullptr;
    const real *El[K];
    real sc[K];
#pragma unroll
    for (int l = 0; l < K; ++l) {
        const int s = min(s0 + l + 1, ch.N);
        El[l] = E + (size_t)ch.types[s - 1] * V;
        sc[l] = pow2_neg<real>(st[r].scale_e[s - 1]);
    }
    auto plane = [&](int idx) { return (unsigned)wrapm(t.z0 - K + idx, R.Lz) * LxLy; };
    // loads of plane iteration `it`: the level-0 plane and every level's field factors
    auto load = [&](int it, real(&fin)[H], real(&ev)[K][H]) {
        const unsigned zi = plane(it);
#pragma unroll
        for (int j = 0; j < H; ++j) fin[j] = Gin ? Gin[zi + yo[j]] : (real)1;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            if (l >= nsteps) break;
            const unsigned zq = plane(it - (l + 1));
#pragma unroll
            for (int j = 0; j < H; ++j) ev[l][j] = El[l][zq + yo[j]];
        }
    };
    real P[K][H], U[K][H], fn[H], en[K][H];
#pragma unroll
    for (int l = 0; l < K; ++l)
#pragma unroll
        for (int j = 0; j < H; ++j) P[l][j] = U[l][j] = en[l][j] = (real)0;
    double gsum[K], esum[2] = {0.0, 0.0};
#pragma unroll
    for (int l = 0; l < K; ++l) gsum[l] = 0.0;
    const int M = t.live ? t.cz + 2 * K : 0;
    if (M > 0) load(0, fn, en);
    for (int i = 0; i < M; ++i) {
        real f[H], e[K][H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            f[j] = fn[j];
#pragma unroll
            for (int l = 0; l < K; ++l) e[l][j] = en[l][j];
        }
        if (i + 1 < M) load(i + 1, fn, en);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            if (l >= nsteps) break;
            const int idx = i - (l + 1);   // plane completed at this level
            real S[H];
            stencil_push<real, H>(f, P[l], U[l], S, c0, c1, c2, c3);
#pragma unroll
            for (int j = 0; j < H; ++j) f[j] = e[l][j] * S[j] * sc[l];
            if (idx >= K && idx < K + t.cz && xcore) {
                const unsigned zq = plane(idx);
                real *Gs = G + (size_t)(s0 + l) * V;
#pragma unroll
                for (int j = K; j < H - K; ++j) {
                    if (j - K >= t.cy) break;
                    Gs[zq + yo[j]] = f[j];
                    gsum[l] += (double)f[j];
                    if (s0 + l == 0 && sums) {
                        esum[0] += (double)E[zq + yo[j]];
                        esum[1] += (double)E[V + zq + yo[j]];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int l = 0; l < K; ++l) {
        if (l >= nsteps) break;
        const int s = s0 + l + 1;
        if (sums || s == ch.N) {
            const double v = block_sum(gsum[l]);
            if (threadIdx.x == 0) partG[(long long)(s - 1) * nblocks + pb] = v;
        }
    }
    if (s0 == 0 && sums) {
        double v = block_sum(esum[0]);
        if (threadIdx.x == 0) partG[(long long)ch.N * nblocks + pb] = v;
        v = block_sum(esum[1]);
        if (threadIdx.x == 0) partG[(long long)(ch.N + 1) * nblocks + pb] = v;
    }
}

// Backward sweep, steps s_hi down to s_hi - nsteps + 1 (nsteps <= K = 2), from
// G+_{s_hi+1} in gin (G+_{N+1} = 1).  Stores G+ of the last level into gout (unless it
// reaches s = 1).  The density terms G_s sigma[G+_{s+1}] of a site are summed per species
// over the launch's levels; a launch that does not reach s = 1 stores the sum for the
// species of its last step s_lo in slot s_lo - 1 and, when its first step s_hi is of the
// other species, that species' term in slot s_hi - 1.  The launch reaching s = 1 adds the
// sums the earlier launches stored (same launch schedule: steps N, N - K, ...) to its own,
// normalises with phibar_p / (N Q) and writes phi (final_mode 0, field layout) or
// g = phi^t - phi (final_mode 1, polymer layout) with block partial sums d.g, g.z, |g_A|^2,
// |g_B|^2 (z = g / phi^t when preconditioned).  Loads are issued a plane iteration ahead.
template <typename real, int K, int H>
__global__ __launch_bounds__(kBlock) void k_bwd_stream(const int *__restrict__ blk_rep,
                                                       const int *__restrict__ blk_first,
                                                       const Rep *__restrict__ rep,
                                                       const RepState *__restrict__ st, Chain ch, int s_hi,
                                                       int nsteps, int cz, PropBufs<real> b,
                                                       const real *__restrict__ gin, real *__restrict__ gout,
                                                       int final_mode, const double *__restrict__ phit,
                                                       const double *__restrict__ d, double *__restrict__ out,
                                                       double *__restrict__ part, ArgReps ar)
{
    static_assert(K == 2, "the pending density sums hold one plane");
    const int pb = plan_block();
    const int r = stream_replica(pb, blk_rep, ar);
    if (!st[r].active && ar.n != 1) return;
    const Rep R = stream_rep(ar, rep, r);
    const int bf = ar.n ? ar.blk_first[r] : blk_first[r];
    const int wv = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const STile<K, H> t = stream_tile<K, H>(R, cz, (pb - bf) * (kBlock / 64) + wv);
    const int N = ch.N;
    const unsigned V = (unsigned)R.V, LxLy = (unsigned)(R.Lx * R.Ly);
    const real c0 = (real)R.c[0], c1 = (real)R.c[1], c2 = (real)R.c[2], c3 = (real)R.c[3];
    real *G = b.G + (long long)N * R.site_off;
    const real *E = b.E + off_poly(R);
    const int x = wrapm(t.x0 - K + lane, R.Lx);
    const bool xcore = lane >= K && lane < K + t.cx;
    unsigned yo[H];
#pragma unroll
    for (int j = 0; j < H; ++j) yo[j] = (unsigned)(wrapm(t.y0 - K + j, R.Ly) * R.Lx + x);
    const real *Gin = s_hi < N ? gin + R.site_off : nullptr;
    const int s_lo = s_hi - nsteps + 1;
    const bool fin = s_lo == 1;
    const int t_lo = ch.types[s_lo - 1], t_hi = ch.types[s_hi - 1];
    const bool mixed = nsteps == 2 && t_hi != t_lo;
    const real *El[K];
    const real *Gsl[K];
    real sc[K];
#pragma unroll
    for (int l = 0; l < K; ++l) {
        const int s = max(s_hi - l, 1);
        El[l] = E + (size_t)ch.types[s - 1] * V;
        Gsl[l] = G + (size_t)(s - 1) * V;
        sc[l] = pow2_neg<real>(st[r].scale_e[s - 1]);
    }
    const double coef = fin ? st[r].phibar_p / ((double)N * st[r].q) : 0.0;
    const long long fo = off_field(R, ch.nsp), po = off_poly(R);
    real *gout_r = gout + R.site_off;
    auto plane = [&](int idx) { return (unsigned)wrapm(t.z0 - K + idx, R.Lz) * LxLy; };
    auto is_core = [&](int idx) { return idx >= K && idx < K + t.cz; };
    // loads of plane iteration `it`: the level-0 plane, the levels' field factors (not
    // needed at s = 1) and, on core planes, the stored G_s of the core rows
    auto load = [&](int it, real(&fin_)[H], real(&ev)[K][H], real(&gv)[K][H]) {
        const unsigned zi = plane(it);
#pragma unroll
        for (int j = 0; j < H; ++j) fin_[j] = Gin ? Gin[zi + yo[j]] : (real)1;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            if (l >= nsteps) break;
            const int idx = it - (l + 1);
            const unsigned zq = plane(idx);
            if (s_hi - l > 1) {
#pragma unroll
                for (int j = 0; j < H; ++j) ev[l][j] = El[l][zq + yo[j]];
            }
            if (is_core(idx)) {
#pragma unroll
                for (int j = K; j < H - K; ++j) gv[l][j] = Gsl[l][zq + yo[j]];
            }
        }
    };
    // pend: the first level's terms of the plane the last level completes in this
    // iteration (formed one iteration earlier); pnew: those of the next plane
    real P[K][H], U[K][H], pend[H], pnew[H], fn[H], en[K][H], gn[K][H];
#pragma unroll
    for (int l = 0; l < K; ++l)
#pragma unroll
        for (int j = 0; j < H; ++j) P[l][j] = U[l][j] = en[l][j] = gn[l][j] = (real)0;
#pragma unroll
    for (int j = 0; j < H; ++j) pend[j] = pnew[j] = (real)0;
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    const int M = t.live ? t.cz + 2 * K : 0;
    if (M > 0) load(0, fn, en, gn);
    for (int i = 0; i < M; ++i) {
        real f[H], e[K][H], gs[K][H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            f[j] = fn[j];
#pragma unroll
            for (int l = 0; l < K; ++l) {
                e[l][j] = en[l][j];
                gs[l][j] = gn[l][j];
            }
        }
        if (i + 1 < M) load(i + 1, fn, en, gn);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            if (l >= nsteps) break;
            const int s = s_hi - l;
            const int idx = i - (l + 1);
            real S[H];
            stencil_push<real, H>(f, P[l], U[l], S, c0, c1, c2, c3);
            const bool core = is_core(idx) && xcore;
            // the density terms of this level at the core rows
            real term[H];
#pragma unroll
            for (int j = 0; j < H; ++j) term[j] = (j >= K && j < H - K) ? gs[l][j] * S[j] : (real)0;
            // G+_s feeds the next level (and, at the last level, the next launch)
            if (s > 1) {
#pragma unroll
                for (int j = 0; j < H; ++j) f[j] = e[l][j] * S[j] * sc[l];
                if (l == nsteps - 1 && core) {
                    const unsigned zq = plane(idx);
#pragma unroll
                    for (int j = K; j < H - K; ++j) {
                        if (j - K >= t.cy) break;
                        gout_r[zq + yo[j]] = f[j];
                    }
                }
            }
            if (!core) continue;
            if (l < nsteps - 1) {   // the site's later level comes in the next plane iteration
#pragma unroll
                for (int j = 0; j < H; ++j) pnew[j] = term[j];
                continue;
            }
            // all of this plane's levels are in: store or finish
            const unsigned zq = plane(idx);
#pragma unroll
            for (int j = K; j < H - K; ++j) {
                if (j - K >= t.cy) break;
                const unsigned site = zq + yo[j];
                // per-species sums of the launch's terms (level 1 pending, then the last)
                real own[2] = {(real)0, (real)0};
                if (nsteps == 2) own[t_hi] += pend[j];
                own[t_lo] += term[j];
                if (!fin) {
                    G[(size_t)(s_lo - 1) * V + site] = own[t_lo];
                    if (mixed) G[(size_t)(s_hi - 1) * V + site] = own[t_hi];
                    continue;
                }
                double a[2] = {0.0, 0.0};
                // the earlier launches' sums, in launch order
                for (int sh = N; sh > s_hi; sh -= K) {
                    const int sl = sh - K + 1;
                    const int ta = ch.types[sl - 1], tb = ch.types[sh - 1];
                    a[ta] += (double)G[(size_t)(sl - 1) * V + site];
                    if (tb != ta) a[tb] += (double)G[(size_t)(sh - 1) * V + site];
                }
                a[0] += (double)own[0];
                a[1] += (double)own[1];
#pragma unroll
                for (int I = 0; I < 2; ++I) {
                    const double ph = coef * a[I];
                    if (final_mode == 0) {
                        out[fo + (long long)I * V + site] = ph;
                    } else {
                        const double tI = phit[fo + (long long)I * V + site];
                        const double gI = tI - ph;
                        out[po + (long long)I * V + site] = gI;
                        if (d) sums[0] += d[po + (long long)I * V + site] * gI;
                        sums[1] += ch.precond ? gI * gI / tI : gI * gI;
                        sums[2 + I] += gI * gI;
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < H; ++j) pend[j] = pnew[j];
    }
    if (fin && final_mode == 1) {
        block_sums(sums);
        if (threadIdx.x == 0)
            for (int q = 0; q < 4; ++q) part[(long long)pb * kNQ + q] = sums[q];
    }
}

// ---- launchers ---------------------------------------------------------------------

template <typename real, int H, int K>
struct StreamKernels {
    static void fwd(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, int s0, int n, int cz,
                    PropBufs<real> b, double *partG, int sums, hipEvent_t e0, hipEvent_t e1)
    {
        if (e0)
            hipExtLaunchKernelGGL((k_fwd_stream<real, K, H>), dim3(p.nblocks), dim3(kBlock), 0, s, e0, e1, 0,
                                  p.blk_rep, p.blk_first, rep, st, ch, s0, n, cz, b, partG, p.nblocks, sums, p.args);
        else
            hipLaunchKernelGGL((k_fwd_stream<real, K, H>), dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep,
                               p.blk_first, rep, st, ch, s0, n, cz, b, partG, p.nblocks, sums, p.args);
    }
    static void bwd(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, int s_hi, int n, int cz,
                    PropBufs<real> b, const real *gin, real *gout, int final_mode, const double *phit,
                    const double *d, double *out, double *part, hipEvent_t e0, hipEvent_t e1)
    {
        if (e0)
            hipExtLaunchKernelGGL((k_bwd_stream<real, K, H>), dim3(p.nblocks), dim3(kBlock), 0, s, e0, e1, 0,
                                  p.blk_rep, p.blk_first, rep, st, ch, s_hi, n, cz, b, gin, gout, final_mode, phit,
                                  d, out, part, p.args);
        else
            hipLaunchKernelGGL((k_bwd_stream<real, K, H>), dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep,
                               p.blk_first, rep, st, ch, s_hi, n, cz, b, gin, gout, final_mode, phit, d, out, part,
                               p.args);
    }
};

template <typename real>
void launch_fwd_stream(const TileCfg &cfg, hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                       int s0, int n, PropBufs<real> b, double *partG, int sums, hipEvent_t e0, hipEvent_t e1)
{
#define HSF_CASE(H, CZ, K)                                                                                  \
    if (cfg.cy == H && cfg.cz == CZ && cfg.k == K)                                                          \
        return StreamKernels<real, H, K>::fwd(s, p, rep, st, ch, s0, n, CZ, b, partG, sums, e0, e1);
    HSF_STREAM_CONFIGS(HSF_CASE)
#undef HSF_CASE
}

template <typename real>
void launch_bwd_stream(const TileCfg &cfg, hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                       int s_hi, int n, PropBufs<real> b, const real *gin, real *gout, int final_mode,
                       const double *phit, const double *d, double *out, double *part, hipEvent_t e0, hipEvent_t e1)
{
#define HSF_CASE(H, CZ, K)                                                                                  \
    if (cfg.cy == H && cfg.cz == CZ && cfg.k == K)                                                          \
        return StreamKernels<real, H, K>::bwd(s, p, rep, st, ch, s_hi, n, CZ, b, gin, gout, final_mode, phit, d, \
                                              out, part, e0, e1);
    HSF_STREAM_CONFIGS(HSF_CASE)
#undef HSF_CASE
}

#define HSF_INST(real)                                                                                        \
    template void launch_fwd_stream<real>(const TileCfg &, hipStream_t, const Plan &, const Rep *, RepState *, \
                                          Chain, int, int, PropBufs<real>, double *, int, hipEvent_t,        \
                                          hipEvent_t);                                                       \
    template void launch_bwd_stream<real>(const TileCfg &, hipStream_t, const Plan &, const Rep *, RepState *, \
                                          Chain, int, int, PropBufs<real>, const real *, real *, int,        \
                                          const double *, const double *, double *, double *, hipEvent_t,    \
                                          hipEvent_t);
HSF_INST(double)
HSF_INST(float)
#undef HSF_INST

}  // namespace hsf
