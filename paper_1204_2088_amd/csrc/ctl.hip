// ctl.hip -- deterministic reductions and the per-replica control of the
// Fletcher-Reeves inversion (section 2: the fields are determined
// self-consistently at every step by nonlinear conjugate gradients).
//
// The inversion minimises the convex objective
//   Phi(w) = (phibar_p V / N) ln Q[w] + phibar_s V ln<exp(-w_S)> + sum_I sum_r phi^t_I w_I,
// whose gradient is phi^t - phi[w].  Line search: secant on h(alpha) = d.grad Phi(w + alpha d)
// from alpha_0 = -(d.g) / sum d^2 phi^t; a trial is accepted when |h| <= 0.1 |h(0)|, after
// three trials, or when the secant slope or the next alpha is not positive (extrapolation
// capped at 8x).  beta = (g_new.z_new) / (g_old.z_old) with z = g, or z = g / phi^t in the
// diagonally preconditioned variant; restart every 50 iterations and whenever the new
// direction would not descend (d_new.g_new = -g_new.z_new + beta d.g_new >= 0).
//
// All vector work is done by site kernels that write per-block partial sums; one block
// per replica then sums its blocks' partials in a fixed order and thread 0 runs the
// replica's scalar logic, so every replica of a batch follows its own iteration.
#include <math.h>

#include "device_common.h"

namespace hsf {

// Nearest integer to log2(m), m > 0 finite, from the binary exponent.
__device__ __forceinline__ long round_log2(double m)
{
    int e = 0;
    const double f = frexp(m, &e);   // m = f 2^e, f in [0.5, 1)
    return f < 0.70710678118654752440 ? e - 1 : e;
}

// Per-step power-of-two scales for the next evaluation.  sums[s] = sum_r of the
// stored G_{s+1} of this evaluation (its mean m_s is relative to the cumulative
// scale used), sums[N], sums[N+1] = sum_r E_A, E_B.  Target: stored means near 1.
// Where a mean is not usable (overflow or underflow) the growth is predicted from
// the mean-field factor <E_{t_s}> csum instead.
__device__ void update_scales(RepState &S, const Chain &ch, const double *sums, double V, double csum)
{
    int cum_old = 0, cum_new = 0;
    for (int s = 0; s < ch.N; ++s) {
        cum_old += S.scale_e[s];
        const double m = sums[s] / V;
        long target;
        if (m > 0.0 && isfinite(m)) {
            target = cum_old + round_log2(m);
        } else {
            const double me = sums[ch.N + ch.types[s]] / V * csum;
            target = cum_new + ((me > 0.0 && isfinite(me)) ? round_log2(me) : 0);
        }
        long e = target - cum_new;
        if (e > 100) e = 100;
        if (e < -100) e = -100;
        S.scale_e[s] = (int)e;
        cum_new += (int)e;
    }
}

__device__ void control(RepState &S, int phase, const Chain &ch, const double *red, const double *gsum,
                        double V, double csum, double tol, int max_iter);
__device__ void reduce_and_control(RepState &S, int r, const int *__restrict__ blk_first, const Rep *__restrict__ rep,
                                   const double *__restrict__ part, int phase, const Chain &ch,
                                   const double *__restrict__ partG, int nblocks, double tol, int max_iter);

// One workgroup of kCtlBlock threads per replica: its reductions are chains of dependent
// load batches, so more wavefronts per row shorten them.
constexpr int kCtlBlock = 1024;

__global__ __launch_bounds__(kCtlBlock) void k_reduce_ctl(const int *__restrict__ blk_first,
                                                       RepState *__restrict__ st, const Rep *__restrict__ rep,
                                                       const double *__restrict__ part, int phase, Chain ch,
                                                       const double *__restrict__ partG, int nblocks,
                                                       double tol, int max_iter, RepState *__restrict__ mirror)
{
    const int r = blockIdx.x;
    // work on an LDS copy of the replica's state: one cooperative load and store instead of
    // a dependent global round trip per field in the scalar logic below
    __shared__ RepState S;
    {
        static_assert(sizeof(RepState) % 4 == 0, "RepState is copied as 32-bit words");
        const int *src = reinterpret_cast<const int *>(&st[r]);
        int *dst = reinterpret_cast<int *>(&S);
        for (int k = threadIdx.x; k < (int)(sizeof(RepState) / 4); k += kCtlBlock) dst[k] = src[k];
    }
    __syncthreads();

    // which replicas take part in this phase (uniform per block)
    bool take;
    switch (phase) {
    case PH_Q: case PH_EVAL0: case PH_TRIAL: case PH_SCALES: take = S.active != 0; break;
    default: take = true; break;
    }
    if (take && phase == PH_BEGIN && !S.pending) {
        take = false;
        __syncthreads();
        if (threadIdx.x == 0) S.accepted = 0;
    }
    if (take) reduce_and_control(S, r, blk_first, rep, part, phase, ch, partG, nblocks, tol, max_iter);
    __syncthreads();
    {
        // the state back to device memory and into the host's pinned mirror, which the
        // host reads after synchronising the stream (no copy launch)
        const int *src = reinterpret_cast<const int *>(&S);
        int *dst = reinterpret_cast<int *>(&st[r]);
        int *hm = mirror ? reinterpret_cast<int *>(&mirror[r]) : nullptr;
        for (int k = threadIdx.x; k < (int)(sizeof(RepState) / 4); k += kCtlBlock) {
            dst[k] = src[k];
            if (hm) hm[k] = src[k];
        }
    }
}

// The reduction of one phase's partial sums for replica r and the scalar control step.
__device__ void reduce_and_control(RepState &S, int r, const int *__restrict__ blk_first, const Rep *__restrict__ rep,
                                   const double *__restrict__ part, int phase, const Chain &ch,
                                   const double *__restrict__ partG, int nblocks, double tol, int max_iter)
{
    const int b0 = blk_first[r], b1 = blk_first[r + 1];
    const double V = (double)rep[r].V;
    __shared__ double vals[kNQ + 66];

    // rows to reduce: nslots slots of `part`, then ng rows of `partG` starting at g_first
    int nslots = 0, g_first = 0, ng = 0;
    switch (phase) {
    case PH_TARGET: nslots = 6; break;
    case PH_EVAL0: nslots = 4; ng = ch.N + 2; break;
    case PH_TRIAL: nslots = 4; break;
    case PH_SCALES: ng = ch.N + 2; break;
    case PH_Q: g_first = ch.N - 1; ng = 1; break;
    case PH_BEGIN: nslots = 2; break;
    case PH_SOLVENT: nslots = 1; break;
    default: break;
    }
    // Each row is split into contiguous parts of the replica's blocks, one wavefront per
    // part (as many parts as the wavefronts allow, the same for every row of the phase);
    // within a part the lanes stride over the blocks and a fixed shuffle tree adds them,
    // then the parts are added in order: the order of additions is fixed, so results are
    // reproducible.
    constexpr int kWaves = kCtlBlock / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nrows = nslots + ng;
    const int parts = nrows > 0 ? (nrows >= kWaves ? 1 : kWaves / nrows) : 1;
    const int span = (b1 - b0 + parts - 1) / parts;
    __shared__ double psum[kWaves];
    for (int t0 = 0; t0 < nrows * parts; t0 += kWaves) {
        const int t = t0 + wid, row = t / parts, pt = t % parts;
        if (row < nrows) {
            const int lo = b0 + pt * span, hi = lo + span < b1 ? lo + span : b1;
            double v = 0.0;
            // unrolled so that the loads of several iterations are in flight together
            if (row < nslots) {
#pragma unroll 8
                for (int b = lo + lane; b < hi; b += 64) v += part[(long long)b * kNQ + row];
            } else {
                const double *base = partG + (long long)(g_first + row - nslots) * nblocks;
#pragma unroll 8
                for (int b = lo + lane; b < hi; b += 64) v += base[b];
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
            if (lane == 0) psum[wid] = v;
        }
        __syncthreads();
        // the rows completed in this round: their parts are the wavefronts t0 .. t0 + kWaves
        if (threadIdx.x < kWaves / parts) {
            const int row = t0 / parts + threadIdx.x;
            if (row < nrows) {
                double v = 0.0;
                for (int q = 0; q < parts; ++q) v += psum[threadIdx.x * parts + q];
                vals[row] = v;
            }
        }
        __syncthreads();
    }
    const double *red = vals;
    const double *gsum = vals + nslots - g_first;   // gsum[s] = sum of stored G_{s+1}
    if (threadIdx.x == 0) control(S, phase, ch, red, gsum, V, rep[r].csum, tol, max_iter);
}

// Scalar logic of one replica after the reductions of a phase (runs in one thread).
__device__ void control(RepState &S, int phase, const Chain &ch, const double *red, const double *gsum,
                        double V, double csum, double tol, int max_iter)
{

    switch (phase) {
    case PH_Q: {
        bool bad;
        q_from_sum(gsum[ch.N - 1], V, S.scale_e, ch.N, S.q, S.ln_q, bad);
        if (bad) S.nonfinite = 1;
        break;
    }
    case PH_TARGET: {
        S.phibar_p = red[0] / V;
        S.phibar_s = red[1] / V;
        S.tnorm2[0] = red[2];
        S.tnorm2[1] = red[3];
        S.wmean[0] = red[4] / V;
        S.wmean[1] = red[5] / V;
        S.tol = tol;
        S.max_iter = max_iter;
        S.active = 1;
        S.done = 0;
        S.pending = 0;
        S.accepted = 0;
        S.iters = 0;
        S.evals = 0;
        S.restarts = 0;
        S.converged = 0;
        S.nonfinite = 0;
        S.trial = 0;
        S.alpha = 0.0;
        S.res = INFINITY;
        break;
    }
    case PH_SCALES: update_scales(S, ch, gsum, V, csum); break;
    case PH_SOLVENT: S.sol_mean = red[0] / V; break;
    case PH_EVAL0: {
        update_scales(S, ch, gsum, V, csum);
        S.evals += 1;
        S.gg = red[1];
        S.res = fmax(sqrt(red[2] / S.tnorm2[0]), sqrt(red[3] / S.tnorm2[1]));
        S.active = 0;
        if (!isfinite(S.res) || S.nonfinite) {
            S.nonfinite = 1;
            S.done = 1;
        } else if (S.res <= S.tol) {
            S.done = 1;
            S.converged = 1;
        } else if (S.max_iter <= 0) {
            S.done = 1;
        } else {
            S.pending = 1;
        }
        break;
    }
    case PH_BEGIN: {
        S.h0 = red[0];
        S.dhd = red[1];
        S.alpha = -S.h0 / S.dhd;
        S.a_prev = 0.0;
        S.h_prev = S.h0;
        S.trial = 1;
        S.active = 1;
        S.accepted = 0;
        S.pending = 0;
        if (!isfinite(S.alpha)) {
            S.nonfinite = 1;
            S.done = 1;
            S.active = 0;
        }
        break;
    }
    case PH_TRIAL: {
        S.evals += 1;
        const double h = red[0];
        bool accept = fabs(h) <= 0.1 * fabs(S.h0) || S.trial >= 3;
        if (!accept) {
            const double slope = (h - S.h_prev) / (S.alpha - S.a_prev);
            if (!(slope > 0.0)) {
                accept = true;
            } else {
                double an = S.alpha - h / slope;
                if (!(an > 0.0)) {
                    accept = true;
                } else {
                    if (an > 8.0 * S.alpha) an = 8.0 * S.alpha;
                    S.a_prev = S.alpha;
                    S.h_prev = h;
                    S.alpha = an;
                    S.trial += 1;
                }
            }
        }
        if (accept) {
            S.active = 0;
            S.accepted = 1;
            S.iters += 1;
            S.res = fmax(sqrt(red[2] / S.tnorm2[0]), sqrt(red[3] / S.tnorm2[1]));
            if (!isfinite(S.res) || S.nonfinite) {
                S.nonfinite = 1;
                S.done = 1;
                S.beta = 0.0;
            } else if (S.res <= S.tol) {
                S.converged = 1;
                S.done = 1;
                S.beta = 0.0;
            } else {
                const double ggn = red[1];
                double beta = ggn / S.gg;
                S.gg = ggn;
                if (S.iters % 50 == 0) {
                    beta = 0.0;
                    S.restarts += 1;
                } else if (-ggn + beta * h >= 0.0) {
                    beta = 0.0;
                    S.restarts += 1;
                }
                S.beta = beta;
                if (S.iters >= S.max_iter) {
                    S.done = 1;
                } else {
                    S.pending = 1;
                }
            }
        }
        break;
    }
    default: break;
    }
}

void launch_reduce_ctl(hipStream_t s, int n_rep, const Plan &p, RepState *st, const Rep *rep,
                       const double *part, int phase, Chain ch, const double *partG, double tol,
                       int max_iter, RepState *mirror)
{
    hipLaunchKernelGGL(k_reduce_ctl, dim3(n_rep), dim3(kCtlBlock), 0, s, p.blk_first, st, rep, part, phase, ch,
                       partG, p.nblocks, tol, max_iter, mirror);
}

// Partial sums of the inversion target: sum of polymer phi^t, sum of phi^t_S,
// |phi^t_A|^2, |phi^t_B|^2, sum of w_A and of w_B.
__global__ __launch_bounds__(kBlock) void k_target_stats(const int *__restrict__ blk_rep,
                                                         const int *__restrict__ blk_first,
                                                         const Rep *__restrict__ rep, Chain ch,
                                                         const double *__restrict__ phit,
                                                         const double *__restrict__ w, double *__restrict__ part)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (i < V) {
        const long long fo = off_field(R, ch.nsp);
        const double a = phit[fo + i], bb = phit[fo + V + i];
        v[0] = a + bb;
        v[1] = ch.nsp == 3 ? phit[fo + 2 * V + i] : 0.0;
        v[2] = a * a;
        v[3] = bb * bb;
        v[4] = w[fo + i];
        v[5] = w[fo + V + i];
    }
    block_sums(v);
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; ++q) part[(long long)plan_block() * kNQ + q] = v[q];
}

void launch_target_stats(hipStream_t s, const Plan &p, const Rep *rep, RepState *, Chain ch,
                         const double *phit, const double *w, double *part)
{
    hipLaunchKernelGGL(k_target_stats, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, ch,
                       phit, w, part);
}

// Local ideal-gas starting guess w_I = -ln phi_I (the constant -ln <phi_I> is removed
// by the gauge shift that follows).
__global__ __launch_bounds__(kBlock) void k_local_guess(const int *__restrict__ blk_rep,
                                                        const int *__restrict__ blk_first,
                                                        const Rep *__restrict__ rep, Chain ch,
                                                        const double *__restrict__ phit, double *__restrict__ w)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    if (i >= V) return;
    const long long fo = off_field(R, ch.nsp);
    for (int I = 0; I < 2; ++I) w[fo + I * V + i] = -log(phit[fo + I * V + i]);
}

void launch_local_guess(hipStream_t s, const Plan &p, const Rep *rep, Chain ch, const double *phit,
                        double *w, double *)
{
    hipLaunchKernelGGL(k_local_guess, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, ch,
                       phit, w);
}

// Gauge shift of the polymer fields to zero mean; closed-form solvent field
// w_S = -ln(phi^t_S / phibar_s).
__global__ __launch_bounds__(kBlock) void k_init_fields(const int *__restrict__ blk_rep,
                                                        const int *__restrict__ blk_first,
                                                        const Rep *__restrict__ rep, const RepState *__restrict__ st,
                                                        Chain ch, const double *__restrict__ phit,
                                                        double *__restrict__ w)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    if (i >= V) return;
    const RepState &S = st[sr.r];
    const long long fo = off_field(R, ch.nsp);
    w[fo + i] -= S.wmean[0];
    w[fo + V + i] -= S.wmean[1];
    if (ch.nsp == 3) w[fo + 2 * V + i] = -log(phit[fo + 2 * V + i] / S.phibar_s);
}

void launch_init_fields(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                        const double *phit, double *w)
{
    hipLaunchKernelGGL(k_init_fields, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, st, ch,
                       phit, w);
}

// Conjugate-gradient vector update, z = g (or g / phi^t when preconditioned).
//   init = 1 (replicas pending their first iteration): d = -z, g from the start evaluation
//   init = 0 (replicas whose trial was accepted): w += alpha d and, unless the replica is
//            done, d = -z + beta d with g the accepted trial's gradient g_trial (read in
//            place: only the scalars of g are needed later, and the next start evaluation
//            rewrites the vector g)
// Partial sums d.g and sum d^2 phi^t for the next alpha_0.
__global__ __launch_bounds__(kBlock) void k_cg_update(const int *__restrict__ blk_rep,
                                                      const int *__restrict__ blk_first,
                                                      const Rep *__restrict__ rep, const RepState *__restrict__ st,
                                                      Chain ch, int init, double *__restrict__ w,
                                                      const double *__restrict__ g, const double *__restrict__ gt,
                                                      double *__restrict__ d, const double *__restrict__ phit,
                                                      double *__restrict__ part)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const RepState &S = st[sr.r];
    if (init ? !S.pending : !S.accepted) return;
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    double dg = 0.0, dhd = 0.0;
    if (i < V) {
        const long long fo = off_field(R, ch.nsp), po = off_poly(R);
        const double alpha = S.alpha, beta = S.beta;
        const bool upd_d = init || !S.done;
#pragma unroll
        for (int I = 0; I < 2; ++I) {
            const long long k = po + I * V + i;
            double gI;
            double dI = d[k];
            if (init) {
                gI = g[k];
            } else {
                w[fo + I * V + i] = fma(alpha, dI, w[fo + I * V + i]);
                gI = gt[k];
            }
            if (upd_d) {
                const double zI = ch.precond ? gI / phit[fo + I * V + i] : gI;
                dI = init ? -zI : fma(beta, dI, -zI);
                d[k] = dI;
            }
            dg += dI * gI;
            dhd += dI * dI * phit[fo + I * V + i];
        }
    }
    double t[2] = {dg, dhd};
    block_sums(t);
    if (threadIdx.x == 0) {
        part[(long long)plan_block() * kNQ + 0] = t[0];
        part[(long long)plan_block() * kNQ + 1] = t[1];
    }
}

void launch_cg_update(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, int init,
                      double *w, double *g, const double *gt, double *d, const double *phit, double *part)
{
    hipLaunchKernelGGL(k_cg_update, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, st, ch,
                       init, w, g, gt, d, phit, part);
}

// Solvent density of eq. 2: pass 0 sums exp(-w_S); pass 1 writes
// phi_S = phibar_s exp(-w_S) / <exp(-w_S)> into the field-layout output.
__global__ __launch_bounds__(kBlock) void k_solvent(const int *__restrict__ blk_rep,
                                                    const int *__restrict__ blk_first,
                                                    const Rep *__restrict__ rep, const RepState *__restrict__ st,
                                                    Chain ch, int pass, const double *__restrict__ w,
                                                    double *__restrict__ out, double *__restrict__ part)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    const long long fo = off_field(R, ch.nsp);
    if (pass == 0) {
        const double v = i < V ? exp(-w[fo + 2 * V + i]) : 0.0;
        const double t = block_sum(v);
        if (threadIdx.x == 0) part[(long long)plan_block() * kNQ] = t;
    } else if (i < V) {
        const RepState &S = st[sr.r];
        out[fo + 2 * V + i] = S.phibar_s * exp(-w[fo + 2 * V + i]) / S.sol_mean;
    }
}

void launch_solvent(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, int pass,
                    const double *w, const double *, double *out, double *part)
{
    hipLaunchKernelGGL(k_solvent, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, st, ch,
                       pass, w, out, part);
}

}  // namespace hsf

namespace hsf {

}  // namespace hsf
