// obs.hip -- observables of a state (w, phi): the free-energy density of eq. 1 on the
// lattice and the order parameters of the melt and the solution.
//
// Free energy (v0 = 1, kT = 1, integrals as site sums, per site):
//   F = -n_p ln(V Q) + ln n_p! - n_s ln(V <exp(-w_S)>) + ln n_s!
//       - sum_I sum_r phi_I w_I + 1/2 sum_IJ chi_IJ sum_r phi_I sigma[phi_J]
//       + kappa/2 sum_r (sum_I phi_I - 1)^2,
// n_p = phibar_p V / N chains, n_s = phibar_s V solvent beads, Q the single-chain
// partition function of the last evaluation and sigma the linkage stencil (the
// interaction kernel whose derivative is the chemical potential of eq. 4).
// Order parameters: S_melt = sqrt(V^-1 sum_r sum_I (phi_I - <phi_I>)^2) and
// S_sol = V^-1 sum_r |phi_A + phi_B - <phi_A> - <phi_B>|.
//
// Two site passes write per-block partial sums; after each, one block per replica
// sums its blocks in a fixed order, so the results are reproducible.
#include <math.h>

#include "device_common.h"

namespace hsf {

namespace {

constexpr int kObsStride = 8;   // doubles per replica in the observables scratch

// pass 0 slots: 0-2 sum phi_I, 3 sum phi.w, 4 interaction, 5 incompressibility
// pass 1 slots: 0 sum_I (phi_I - <phi_I>)^2, 1 |phi_A + phi_B - <phi_A> - <phi_B>|
__global__ __launch_bounds__(kBlock) void k_obs_sites(const int *__restrict__ blk_rep,
                                                      const int *__restrict__ blk_first,
                                                      const Rep *__restrict__ rep, Chain ch, int pass,
                                                      const double *__restrict__ w,
                                                      const double *__restrict__ phi,
                                                      const double *__restrict__ mean,
                                                      double *__restrict__ part)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    const int nsp = ch.nsp;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (i < V) {
        const long long fo = off_field(R, nsp);
        const double *p = phi + fo;
        if (pass == 0) {
            const int x = (int)(i % R.Lx), y = (int)((i / R.Lx) % R.Ly), z = (int)(i / ((long long)R.Lx * R.Ly));
            double tot = 0.0, inter = 0.0, pw = 0.0;
            double sig[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int J = 0; J < 3; ++J)
                if (J < nsp)
                    sig[J] = stencil27<double>(p + J * V, x, y, z, R.Lx, R.Ly, R.Lz, R.c[0], R.c[1], R.c[2], R.c[3]);
#pragma unroll
            for (int I = 0; I < 3; ++I) {
                if (I >= nsp) break;
                const double pI = p[I * V + i];
                v[I] = pI;
                tot += pI;
                pw += pI * w[fo + I * V + i];
                double cs = 0.0;
#pragma unroll
                for (int J = 0; J < 3; ++J)
                    if (J < nsp) cs += R.chi[I][J] * sig[J];
                inter += pI * cs;
            }
            v[3] = pw;
            v[4] = 0.5 * inter;
            v[5] = 0.5 * R.kappa * (tot - 1.0) * (tot - 1.0);
        } else {
            const double *m = mean + (long long)sr.r * kObsStride;
            double sq = 0.0;
#pragma unroll
            for (int I = 0; I < 3; ++I) {
                if (I >= nsp) break;
                const double d = p[I * V + i] - m[I];
                sq += d * d;
            }
            v[0] = sq;
            v[1] = fabs(p[i] + p[V + i] - m[0] - m[1]);
        }
    }
    const int nslots = pass == 0 ? 6 : 2;   // uniform over the grid
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (q >= nslots) break;
        const double t = block_sum(v[q]);
        if (threadIdx.x == 0) part[(long long)plan_block() * kNQ + q] = t;
    }
}

// One block per replica: fixed-order sums of the partials.  Pass 0 stores the
// species means and the three energy sums; pass 1 combines everything into
// out[r] = {F / V, S_melt, S_sol}.
__global__ __launch_bounds__(kBlock) void k_obs_reduce(const int *__restrict__ blk_first,
                                                       const Rep *__restrict__ rep,
                                                       const RepState *__restrict__ st, Chain ch, int pass,
                                                       const double *__restrict__ part,
                                                       double *__restrict__ scratch, double *__restrict__ out)
{
    const int r = blockIdx.x;
    const int b0 = blk_first[r], b1 = blk_first[r + 1];
    const double V = (double)rep[r].V;
    __shared__ double red[kNQ];
    const int nslots = pass == 0 ? 6 : 2;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int row = wid; row < nslots; row += kBlock / 64) {
        double v = 0.0;
        for (int b = b0 + lane; b < b1; b += 64) v += part[(long long)b * kNQ + row];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) red[row] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double *m = scratch + (long long)r * kObsStride;
    if (pass == 0) {
        for (int I = 0; I < 3; ++I) m[I] = red[I] / V;
        m[3] = red[3];
        m[4] = red[4];
        m[5] = red[5];
        return;
    }
    const RepState &S = st[r];
    const double np = S.phibar_p * V / (double)ch.N;
    double F = -np * (log(V) + S.ln_q) + lgamma(np + 1.0);
    if (ch.nsp == 3) {
        const double ns = S.phibar_s * V;
        F += -ns * log(V * S.sol_mean) + lgamma(ns + 1.0);
    }
    F += -m[3] + m[4] + m[5];
    out[3 * r + 0] = F / V;
    out[3 * r + 1] = sqrt(red[0] / V);
    out[3 * r + 2] = red[1] / V;
}

}  // namespace

void launch_observables(hipStream_t s, const Plan &p, int n_rep, const Rep *rep, const RepState *st, Chain ch,
                        const double *w, const double *phi, double *part, double *scratch, double *out)
{
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_obs_sites, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, ch,
                           pass, w, phi, (const double *)scratch, part);
        hipLaunchKernelGGL(k_obs_reduce, dim3(n_rep), dim3(kBlock), 0, s, p.blk_first, rep, st, ch, pass,
                           (const double *)part, scratch, out);
    }
}

size_t observables_scratch_doubles(int n_rep) { return (size_t)n_rep * (kObsStride + 3); }

// ---- per-step record: each species' amount and the largest flow speed ----

// Slots 0-2: sum over the block's sites of phi_I; slot 3: the block's largest |u|^2
// (0 without a velocity field).
__global__ __launch_bounds__(kBlock) void k_step_sites(const int *__restrict__ blk_rep,
                                                       const int *__restrict__ blk_first,
                                                       const Rep *__restrict__ rep, int nsp,
                                                       const double *__restrict__ phi,
                                                       const double *__restrict__ u, double *__restrict__ part)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    double v[3] = {0.0, 0.0, 0.0}, u2 = 0.0;
    if (i < V) {
        const double *p = phi + off_field(R, nsp);
#pragma unroll
        for (int I = 0; I < 3; ++I)
            if (I < nsp) v[I] = p[I * V + i];
        if (u) {
            const double *uu = u + 3 * R.site_off;
            const double a = uu[i], b = uu[V + i], c = uu[2 * V + i];
            u2 = a * a + b * b + c * c;
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double t = block_sum(v[q]);
        if (threadIdx.x == 0) part[(long long)plan_block() * kNQ + q] = t;
    }
    __shared__ double wm[kBlock / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) u2 = fmax(u2, __shfl_down(u2, o, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = u2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
#pragma unroll
        for (int k = 0; k < kBlock / 64; ++k) m = fmax(m, wm[k]);
        part[(long long)plan_block() * kNQ + 3] = m;
    }
}

// One block per replica: out[4 r + I] = sum of phi_I (blocks in order), out[4 r + 3] = max |u|.
__global__ __launch_bounds__(64) void k_step_reduce(const int *__restrict__ blk_first,
                                                    const double *__restrict__ part, double *__restrict__ out)
{
    const int r = blockIdx.x, lane = threadIdx.x;
    const int b0 = blk_first[r], b1 = blk_first[r + 1];
    double s[3] = {0.0, 0.0, 0.0}, m = 0.0;
    for (int b = b0 + lane; b < b1; b += 64) {
#pragma unroll
        for (int q = 0; q < 3; ++q) s[q] += part[(long long)b * kNQ + q];
        m = fmax(m, part[(long long)b * kNQ + 3]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int q = 0; q < 3; ++q) s[q] += __shfl_down(s[q], o, 64);
        m = fmax(m, __shfl_down(m, o, 64));
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) out[4 * r + q] = s[q];
        out[4 * r + 3] = sqrt(m);
    }
}

void launch_step_moments(hipStream_t s, const Plan &p, int n_rep, const Rep *rep, int nsp, const double *phi,
                         const double *u, double *part, double *out)
{
    hipLaunchKernelGGL(k_step_sites, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, nsp, phi, u,
                       part);
    hipLaunchKernelGGL(k_step_reduce, dim3(n_rep), dim3(64), 0, s, p.blk_first, (const double *)part, out);
}

}  // namespace hsf
