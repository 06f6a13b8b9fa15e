// prop.hip -- chain-propagator sweeps of the SCF density functional
// (eq. 16-17): field preparation, forward sweep, backward sweep with density
// accumulation and the final normalisation (eq. 2).
//
// Storage scheme: every forward propagator G_s (s = 1..N) is stored; the
// backward propagator lives in two ping-pong planes.  Each step divides by a
// per-step power of two 2^e_s (exact), the same e_s in both sweeps, which keeps
// FP32 propagators in range while leaving densities unchanged:
//   stored G_s  = G_s / 2^(e_1 + .. + e_s)
//   stored G+_s = G+_s * 2^(e_1 + .. + e_{s-1}) / 2^(e_1 + .. + e_N)
// so G_s sigma[G+_{s+1}] carries the single factor 2^-(e_1+..+e_N), which
// cancels against the same factor in the stored Q.
#include "device_common.h"

namespace hsf {

template <typename real>
__device__ __forceinline__ real pow2_neg(int e)
{
    return (real)ldexp(1.0, -e);
}

// Field preparation (E = exp(-w') with w' = w, or w + alpha d for a line-search
// trial), first forward step G_1 = E_{t_1} sigma[1] / 2^e_1, zeroed accumulators.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_prep(const int *__restrict__ blk_rep,
                                                 const int *__restrict__ blk_first,
                                                 const Rep *__restrict__ rep, const RepState *__restrict__ st,
                                                 Chain ch, const double *__restrict__ w,
                                                 const double *__restrict__ d, int use_alpha,
                                                 PropBufs<real> b, double *__restrict__ acc,
                                                 double *__restrict__ partG, int nblocks)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    if (!st[sr.r].active) return;
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    double gsum = 0.0, esum[2] = {0.0, 0.0};
    if (i < V) {
        const long long fo = off_field(R, ch.nsp), po = off_poly(R);
        const double alpha = st[sr.r].alpha;
        real e[2];
#pragma unroll
        for (int I = 0; I < 2; ++I) {
            double x = w[fo + I * V + i];
            if (use_alpha) x = fma(alpha, d[po + I * V + i], x);
            e[I] = (real)exp(-x);
            b.E[po + I * V + i] = e[I];
            acc[po + I * V + i] = 0.0;
        }
        const real g1 = e[ch.types[0]] * (real)R.csum * pow2_neg<real>(st[sr.r].scale_e[0]);
        b.G[(long long)ch.N * R.site_off + i] = g1;
        gsum = (double)g1;
        esum[0] = (double)e[0];
        esum[1] = (double)e[1];
    }
    double t = block_sum(gsum);
    if (threadIdx.x == 0) partG[blockIdx.x] = t;
    // sums of E per species (rows N and N+1): mean-field fallback for the scales
    t = block_sum(esum[0]);
    if (threadIdx.x == 0) partG[(long long)ch.N * nblocks + blockIdx.x] = t;
    t = block_sum(esum[1]);
    if (threadIdx.x == 0) partG[(long long)(ch.N + 1) * nblocks + blockIdx.x] = t;
}

// Forward step s >= 2: G_s = E_{t_s} sigma[G_{s-1}] / 2^e_s.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_fwd(const int *__restrict__ blk_rep,
                                                const int *__restrict__ blk_first,
                                                const Rep *__restrict__ rep, const RepState *__restrict__ st,
                                                Chain ch, int s, PropBufs<real> b,
                                                double *__restrict__ partG, int nblocks)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    if (!st[sr.r].active) return;
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    double gsum = 0.0;
    if (i < V) {
        const int x = (int)(i % R.Lx);
        const int y = (int)((i / R.Lx) % R.Ly);
        const int z = (int)(i / ((long long)R.Lx * R.Ly));
        const long long go = (long long)ch.N * R.site_off;
        const real *in = b.G + go + (long long)(s - 2) * V;
        const real S = stencil27<real>(in, x, y, z, R.Lx, R.Ly, R.Lz, (real)R.c[0], (real)R.c[1],
                                       (real)R.c[2], (real)R.c[3]);
        const real g = b.E[off_poly(R) + ch.types[s - 1] * V + i] * S * pow2_neg<real>(st[sr.r].scale_e[s - 1]);
        b.G[go + (long long)(s - 1) * V + i] = g;
        gsum = (double)g;
    }
    const double t = block_sum(gsum);
    if (threadIdx.x == 0) partG[(long long)(s - 1) * nblocks + blockIdx.x] = t;
}

// Backward step s (N down to 1): S = sigma[G+_{s+1}] (G+_{N+1} = 1),
// acc_{t_s} += G_s S, G+_s = E_{t_s} S / 2^e_s.  At s = 1 the densities are
// normalised, phi_I = phibar_p / (N Q) acc_I, and written as densities
// (final_mode 0, field layout) or as the gradient g = phi^t - phi with its dot
// products (final_mode 1, polymer layout; partial sums d.g, g.g, |g_A|^2, |g_B|^2).
template <typename real>
__global__ __launch_bounds__(kBlock) void k_bwd(const int *__restrict__ blk_rep,
                                                const int *__restrict__ blk_first,
                                                const Rep *__restrict__ rep, const RepState *__restrict__ st,
                                                Chain ch, int s, PropBufs<real> b, double *__restrict__ acc,
                                                int final_mode, const double *__restrict__ phit,
                                                const double *__restrict__ d, double *__restrict__ out,
                                                double *__restrict__ part)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    if (!st[sr.r].active) return;
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    const int N = ch.N;
    const int ts = ch.types[s - 1];
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < V) {
        const long long po = off_poly(R);
        const real *gin = b.Gp[(N - s - 1) & 1] + R.site_off;
        real *gout = b.Gp[(N - s) & 1] + R.site_off;
        real S;
        if (s == N) {
            S = (real)R.csum;
        } else {
            const int x = (int)(i % R.Lx);
            const int y = (int)((i / R.Lx) % R.Ly);
            const int z = (int)(i / ((long long)R.Lx * R.Ly));
            S = stencil27<real>(gin, x, y, z, R.Lx, R.Ly, R.Lz, (real)R.c[0], (real)R.c[1], (real)R.c[2],
                                (real)R.c[3]);
        }
        const real Gs = b.G[(long long)N * R.site_off + (long long)(s - 1) * V + i];
        const double term = (double)Gs * (double)S;
        if (s > 1) {
            acc[po + ts * V + i] += term;
            gout[i] = b.E[po + ts * V + i] * S * pow2_neg<real>(st[sr.r].scale_e[s - 1]);
        } else {
            double a[2] = {acc[po + i], acc[po + V + i]};
            a[ts] += term;
            const double coef = st[sr.r].phibar_p / ((double)N * st[sr.r].q);
            const long long fo = off_field(R, ch.nsp);
#pragma unroll
            for (int I = 0; I < 2; ++I) {
                const double ph = coef * a[I];
                if (final_mode == 0) {
                    out[fo + I * V + i] = ph;
                } else {
                    const double gI = phit[fo + I * V + i] - ph;
                    out[po + I * V + i] = gI;
                    sums[0] += d ? d[po + I * V + i] * gI : 0.0;
                    sums[1] += gI * gI;
                    sums[2 + I] = gI * gI;
                }
            }
        }
    }
    if (s == 1 && final_mode == 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double t = block_sum(sums[q]);
            if (threadIdx.x == 0) part[(long long)blockIdx.x * kNQ + q] = t;
        }
    }
}

template <typename real>
void launch_prep(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, const double *w,
                 const double *d, int use_alpha, PropBufs<real> b, double *acc, double *partG)
{
    hipLaunchKernelGGL(k_prep<real>, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, st,
                       ch, w, d, use_alpha, b, acc, partG, p.nblocks);
}

template <typename real>
void launch_fwd(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, int step,
                PropBufs<real> b, double *partG)
{
    hipLaunchKernelGGL(k_fwd<real>, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, st,
                       ch, step, b, partG, p.nblocks);
}

template <typename real>
void launch_bwd(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, int step,
                PropBufs<real> b, double *acc, int final_mode, const double *phit, const double *d,
                double *out, double *part)
{
    hipLaunchKernelGGL(k_bwd<real>, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, st,
                       ch, step, b, acc, final_mode, phit, d, out, part);
}

#define HSF_INSTANTIATE(real)                                                                          \
    template void launch_prep<real>(hipStream_t, const Plan &, const Rep *, RepState *, Chain,          \
                                    const double *, const double *, int, PropBufs<real>, double *,    \
                                    double *);                                                         \
    template void launch_fwd<real>(hipStream_t, const Plan &, const Rep *, RepState *, Chain, int,      \
                                   PropBufs<real>, double *);                                          \
    template void launch_bwd<real>(hipStream_t, const Plan &, const Rep *, RepState *, Chain, int,      \
                                   PropBufs<real>, double *, int, const double *, const double *,      \
                                   double *, double *);
HSF_INSTANTIATE(double)
HSF_INSTANTIATE(float)
#undef HSF_INSTANTIATE

}  // namespace hsf
