// hsf_internal.h -- shared definitions of the HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hsf.h"

namespace hsf {

constexpr int kBlock = 256;   // threads per block of every site kernel (4 wavefronts)
constexpr int kNQ = 8;        // reduction slots per block in the partials buffer

// Per-replica geometry and parameters, device resident (read-only in kernels).
struct Rep {
    int Lx, Ly, Lz, hydro;
    long long V;            // Lx * Ly * Lz
    long long site_off;     // first site of this replica in the concatenated site space
    double c[4];            // stencil class weights: centre, face, edge, corner
    double csum;            // c0 + 6 c1 + 12 c2 + 8 c3 (sigma applied to a constant 1)
    double chi[3][3];
    double kappa, dt, tau;
    int lb_mode;            // HSF_LB_BGK or HSF_LB_MRT
    double gamma_s, gamma_b, gamma_ghost;
    double omega;           // noise scaling parameter Omega (noise kernels only)
    unsigned long long seed;  // generator key word 0 (word 1 is the replica index)
};

// Per-replica scalars of an evaluation and of the conjugate-gradient inversion.
// FP64, device resident; written only by the one-block-per-replica control kernel.
struct RepState {
    double phibar_p, phibar_s;   // copolymer and solvent amounts of the target
    double tnorm2[2];            // |phi^t_A|^2, |phi^t_B|^2
    double wmean[2];             // mean of w_A, w_B before the gauge shift
    double q;                    // stored-scale Q of the last evaluation
    double ln_q;                 // ln Q including the per-step power-of-two scales
    double alpha, a_prev, h_prev, h0, gg, dhd, beta;
    double res, tol;
    double sol_mean;             // <exp(-w_S)> for the solvent closed form
    int trial, iters, evals, restarts;
    int max_iter;
    int active;                  // evaluation kernels process this replica
    int accepted;                // a trial point was accepted in this iteration
    int pending;                 // waiting for the start of its next iteration
    int done;                    // inversion finished (converged or max_iter)
    int converged;
    int nonfinite;
    int scale_e[64];             // per-step power-of-two exponents e_s (G_s /= 2^e_s)
};

// The replicas of a small batch by value: the hot kernels take them as kernel arguments,
// so a block finds its replica and geometry without dependent loads from device memory
// before its first data load (each such load costs a trip to the last-level cache at
// the start of a kernel).  Larger batches read the tables in device memory.
constexpr int kArgReps = 4;
struct ArgReps {
    int n;                       // replicas, or 0 when the batch is larger than kArgReps
    int blk_first[kArgReps + 1]; // first block of each replica in the plan
    Rep rep[kArgReps];
};

// Launch plan of a site kernel: each block covers kBlock consecutive sites of one replica.
struct Plan {
    int nblocks = 0;
    int *blk_rep = nullptr;      // device: replica of each block
    int *blk_first = nullptr;    // device: first block of each replica, n_rep + 1 entries
    int n_rep = 0;
    ArgReps args{};              // the batch by value when n_rep <= kArgReps
};

// Fill p.args from the host copies of the replicas and the plan's block offsets.
inline void set_plan_args(Plan &p, const Rep *reps, int n_rep, const int *blk_first_host)
{
    p.args = ArgReps{};
    if (n_rep > kArgReps) return;
    p.args.n = n_rep;
    for (int r = 0; r < n_rep; ++r) p.args.rep[r] = reps[r];
    for (int r = 0; r <= n_rep; ++r) p.args.blk_first[r] = blk_first_host[r];
}

// Chain architecture passed by value to kernels.
struct Chain {
    int N;
    int nsp;                     // 2 or 3 species
    int precond;                 // inversion preconditioned by diag(phi^t)
    int types[64];
};

// Kernel-side view of the per-replica layouts.
__host__ __device__ inline long long off_field(const Rep &R, int nsp) { return (long long)nsp * R.site_off; }
__host__ __device__ inline long long off_poly(const Rep &R) { return 2LL * R.site_off; }

// --- launchers (one translation unit per family) --------------------------------

// propagators: FP64 (real = double) and FP32 (real = float) instantiations
template <typename real>
struct PropBufs {
    real *E;        // [rep][2][V]   exp(-w) of the polymer species
    real *G;        // [rep][N][V]   stored forward propagators G_1..G_N
    real *Gp[2];    // [rep][V] x 2  ping-pong backward propagators
};

// reductions and control
enum Phase {
    PH_Q = 0,        // Q of the forward sweep (partials slot 0 of the G_N step)
    PH_TARGET = 1,   // target amounts and norms, field means
    PH_EVAL0 = 2,    // residual at the starting point
    PH_BEGIN = 3,    // start of an iteration: alpha_0 from d.g and d H d
    PH_TRIAL = 4,    // a trial point of the line search
    PH_SCALES = 5,   // update of the per-step scales from the G_s means
    PH_SOLVENT = 6   // <exp(-w_S)>
};
// The control kernel also writes every replica's state into `mirror` (pinned host
// memory, or null), which the host reads after synchronising the stream.
void launch_reduce_ctl(hipStream_t s, int n_rep, const Plan &p, RepState *st, const Rep *rep,
                       const double *part, int phase, Chain ch, const double *partG, double tol,
                       int max_iter, RepState *mirror);

void launch_target_stats(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                         const double *phit, const double *w, double *part);
void launch_local_guess(hipStream_t s, const Plan &p, const Rep *rep, Chain ch, const double *phit,
                        double *w, double *part);
void launch_init_fields(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                        const double *phit, double *w);
void launch_cg_update(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, int init,
                      double *w, double *g, const double *gt, double *d, const double *phit,
                      double *part);
void launch_solvent(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, int pass,
                    const double *w, const double *phi, double *out, double *part);

// dynamics
void launch_mu(hipStream_t s, const Plan &p, const Rep *rep, Chain ch, const double *phi,
               const double *w, double *mu);
void launch_force(hipStream_t s, const Plan &p, const Rep *rep, Chain ch, const double *phi,
                  const double *mu, double *f);
// noise: draw the thermal noise of this step (eq. 13 for LB, eq. 5 for CD) with
// generator step word `step`
// lb_mode: the collision of every replica (HSF_LB_BGK or HSF_LB_MRT), or -1 when mixed
// f32: populations stored as FP32 deviations n_i - w_i from the rest state (else FP64 n_i)
void launch_lb(hipStream_t s, const Plan &p, const Rep *rep, const void *nsrc, void *ndst, bool f32,
               const double *f, double *rho, double *u, bool noise, unsigned long long step, int lb_mode,
               hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, int *bad = nullptr);
// FP64 populations (field layout of the boundary) to the FP32 deviation storage, or back
void launch_lb_convert(hipStream_t s, const Plan &p, const Rep *rep, bool to_f32, const void *src, void *dst);
// bad (may be null): set to 1 by the LB and CD kernels when a moment or an updated density is
// not finite (so that a coupled step can be rolled back)
// noise_flux: scratch for the composition noise's bond fluxes (3 nsp T doubles), or null
// for no noise; diff_scale multiplies dt in the diffusive flux (1/2 in the CN step)
void launch_cd(hipStream_t s, const Plan &p, const Rep *rep, Chain ch, const double *phi,
               const double *mu, const double *u, double *phi_out, double *noise_flux, unsigned long long step,
               hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, double diff_scale = 1.0, int *bad = nullptr);
void launch_lb_rest(hipStream_t s, const Plan &p, const Rep *rep, void *n, bool f32);

// vector kernels of the Crank-Nicolson Newton-Krylov solve (cn.hip); vectors of n doubles
constexpr int kMaxKrylov = 64;
int vec_dot_blocks();
// out[j] = <V_j, x> for j < k (V: k vectors of n doubles); part: k * vec_dot_blocks() doubles
void launch_dots(hipStream_t s, const double *V, int k, long long n, const double *x, double *part, double *out);
// y += scale sum_j coef[j] V_j (coef: k doubles in device memory)
void launch_multi_axpy(hipStream_t s, double *y, const double *V, int k, long long n, const double *coef,
                       double scale);
// out = a x + b y
void launch_lincomb(hipStream_t s, double *out, double a, const double *x, double b, const double *y, long long n);
// F = p - (half - p) - rhs
void launch_cn_residual(hipStream_t s, double *F, const double *p, const double *half, const double *rhs,
                        long long n);

// observables: the free-energy density and order parameters of (w, phi) into
// out[3 r .. 3 r + 2]; uses the Q, phibar and <exp(-w_S)> of the last evaluation in st.
// scratch holds observables_scratch_doubles(n_rep) doubles (out may point into its tail).
void launch_observables(hipStream_t s, const Plan &p, int n_rep, const Rep *rep, const RepState *st, Chain ch,
                        const double *w, const double *phi, double *part, double *scratch, double *out);
size_t observables_scratch_doubles(int n_rep);
// Per replica r: out[4 r + I] = site sum of phi_I (I < nsp, else 0), out[4 r + 3] = max |u|
// (0 when u is null); part holds kNQ doubles per plan block.
void launch_step_moments(hipStream_t s, const Plan &p, int n_rep, const Rep *rep, int nsp, const double *phi,
                         const double *u, double *part, double *out);

}  // namespace hsf

struct hsf_net;
namespace hsf {
int net_predict(hsf_net *n, hipStream_t s, const float *x, int in_ch, int B, int L, float *pred);
int net_channels(const hsf_net *n, int *in_ch, int *out_ch, int *box_multiple);
void net_warm_input(hipStream_t s, const double *phi, const double *h0, const double *h1, int nsp, long long V,
                    int mode, double *part, int max_parts, double *rms, float *x);
void net_warm_apply(hipStream_t s, double *w, const float *p, long long V, int mode, const double *rms,
                    const double *wh0, const double *wh1);
void net_shift_fields(hipStream_t s, double *w, const double *wh0, const double *wh1, long long n);
}  // namespace hsf
