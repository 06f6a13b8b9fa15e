/*
 * hsf.h -- C ABI of the MI355X (gfx950) library for the hybrid
 * lattice-Boltzmann / dynamic self-consistent-field (SCF) method of Zhang,
 * Sevink and Schmid (arXiv:1204.2088).
 *
 * The library computes, on one GPU:
 *   - the SCF density functional phi[w] through chain propagators
 *     (section 2, eq. 2, eq. 16-17; 27-point linkage stencil);
 *   - the self-consistent fields w[phi] by Fletcher-Reeves nonlinear
 *     conjugate gradients (section 2, text after eq. 17);
 *   - the chemical potential and thermodynamic force (eq. 4, eq. 8);
 *   - one D3Q19 lattice-Boltzmann collide-and-stream step (eq. 9-11, with
 *     the single-relaxation-time collision and its forcing term, or the
 *     multiple-relaxation-time collision of eq. 12-14 in the basis of Table 1);
 *   - one conservative update of the convection-diffusion equation (eq. 3),
 *     explicit or with Crank-Nicolson diffusion (section 2);
 *   - the coupled step that alternates the two at equal time steps;
 *   - thermal noise in both parts (eq. 5 and eq. 13), the free-energy density
 *     of eq. 1 and the order parameters, and checkpoints of the run's state;
 *   - a learned warm start for the inversion (a 3-D convolutional network with
 *     its training kernels; not part of the paper).
 *
 * Units: lattice spacing h = 1, kT = 1, the diffusive time unit of the
 * paper; the LB step equals the diffusive step dt.
 *
 * Batching: one context holds n_rep independent replicas ("runs"), each with
 * its own box and parameters but the same chain architecture and precision.
 * Every phase of every call covers all replicas in one kernel launch.
 *
 * Array layouts (all FP64 at this boundary whatever the internal precision):
 *   site index i = x + Lx (y + Ly z), x fastest, periodic boxes;
 *   field arrays (w, phi, mu): replicas one after another, each
 *       [n_species][Lz][Ly][Lx] with species order A, B, then S if present;
 *       replica r starts at element hsf_field_offset(ctx, r);
 *   LB populations: per replica [19][Lz][Ly][Lx], start at 19 * site offset;
 *   vector fields (u, force): per replica [3][Lz][Ly][Lx];
 *   scalar fields (rho): per replica [Lz][Ly][Lx], start at site offset.
 * The D3Q19 velocity order is: rest; +x, -x, +y, -y, +z, -z;
 *   (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1),
 *   (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).
 *
 * Pointers: every data argument is either a host pointer (where = HSF_HOST;
 * the call copies synchronously) or a device pointer on the context's GPU
 * (where = HSF_DEVICE; the copy is ordered on the context's stream).  The
 * caller owns the buffers it passes; the library never keeps them past the
 * call.  The library owns all of its internal device memory.
 *
 * Errors: every int-returning call returns HSF_OK (0) or a negative code;
 * hsf_last_error() gives a message.  A context is not thread safe; distinct
 * contexts are independent.
 */
#ifndef HSF_H
#define HSF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HSF_MAX_BEADS 64
/* Largest box of one replica, Lx * Ly * Lz sites (site indices within a replica are
 * 32-bit); hsf_create refuses larger boxes with HSF_EINVAL.  The replicas of a context
 * together may hold more. */
#define HSF_MAX_SITES 2147483647LL

enum {
    HSF_OK = 0,
    HSF_EINVAL = -1,      /* bad argument; nothing was changed                 */
    HSF_ENOMEM = -2,      /* device allocation failed                           */
    HSF_EHIP = -3,        /* HIP runtime error; message has the HIP string      */
    HSF_ENOCONV = -4,     /* inversion hit max_iter; the iterate is kept        */
    HSF_ENONFINITE = -5   /* a NaN/Inf appeared; hsf_step leaves the state of   */
                          /* the failing step's start (see hsf_step)            */
};

enum { HSF_HOST = 0, HSF_DEVICE = 1 };

/* Precision of the propagators (E = exp(-w), G_s, G+_s).  Reductions (Q,
 * dot products, residual), the density normalisation, the fields and all
 * other arithmetic stay FP64 in both modes.  With HSF_FP32 the LB populations are
 * also stored in FP32, as their deviations n_i - w_i from the rest state (arithmetic
 * in FP64, 180 instead of 360 bytes of traffic per site and step); hsf_set_lb and
 * hsf_get_lb still take FP64 values. */
enum { HSF_FP64 = 0, HSF_FP32 = 1 };

/* Starting guess of an inversion. */
enum {
    HSF_WARM_CURRENT = 0,   /* the fields currently held (previous step's result)   */
    HSF_WARM_LOCAL = 1,     /* local ideal-gas guess w_I = -ln(phi_I / <phi_I>)     */
    HSF_WARM_EXTRAP = 2,    /* w + w^n - w^(n-1): linear extrapolation from the     */
                            /* previous two inversions' results                     */
    HSF_WARM_NET = 3,       /* polymer fields = net(phi) (network with nsp inputs)  */
    HSF_WARM_NET_DELTA = 4, /* w + r net(phi^n, (phi - phi^n) / r)                  */
    HSF_WARM_NET_EXTRAP = 5 /* w + w^n - w^(n-1)                                    */
                            /*   + r net(phi^n, (phi - 2 phi^n + phi^(n-1)) / r)    */
};
/* In the warm starts, w are the fields held, phi the target densities of the new
 * inversion, w^n, phi^n (w^(n-1), phi^(n-1)) the converged fields and targets of
 * the latest (the one before) inversion, and r the rms over species and sites of
 * the density difference fed to the network.  NET_DELTA and NET_EXTRAP take a
 * network with 2 nsp inputs and 2 outputs that predicts the field change per unit
 * density change (the linear response of the inversion).  Modes that lack history
 * fall back: NET_EXTRAP to NET_DELTA after one inversion, NET_DELTA and EXTRAP to
 * the current fields.  hsf_set_fields clears the history. */

typedef struct {
    int Lx, Ly, Lz;              /* periodic box of this replica               */
    int n_beads;                 /* N, beads per copolymer chain (<= 64)       */
    int types[HSF_MAX_BEADS];    /* species of bead s = 1..N at [s-1]: 0 A, 1 B */
    int has_solvent;             /* 1: monomeric solvent S (species 2)         */
    double a;                    /* statistical segment length; when stencil[] */
                                 /* is all zero the weights are the tensor      */
                                 /* product of [al, 1-2al, al], al = a^2/6      */
    double stencil[4];           /* linkage weights: centre, face, edge, corner */
                                 /* (must sum to 1 over the 27 offsets)         */
    double chi[3][3];            /* Flory-Huggins chi_IJ, symmetric, zero diag  */
    double kappa;                /* Helfand parameter kappa_H v0 / kT           */
    double dt;                   /* time step (diffusive units) = LB step       */
    double tau;                  /* LB single relaxation time (> 1/2)           */
    int hydro;                   /* 1: LB flow convects the densities           */
    int precision;               /* HSF_FP64 or HSF_FP32 (same for all replicas) */
    int lb_mode;                 /* HSF_LB_BGK (tau) or HSF_LB_MRT (gammas)     */
    double gamma_s, gamma_b;     /* MRT: eigenvalues of the shear (modes 5-9)   */
                                 /* and bulk (mode 4) stress relaxation, in     */
                                 /* (-1, 1): nu = (1 + gamma_s)/(6 (1 - gamma_s)) */
    double gamma_ghost;          /* MRT: the kinetic (ghost) modes 10-18         */
} hsf_params;

/* LB collision: BGK with the forcing of eq. 14 at every rate 1 - 1/tau, or the
 * multiple-relaxation-time scheme of eq. 12-14 in the basis of Table 1 with the
 * independent eigenvalues gamma_s, gamma_b, gamma_ghost (conserved modes 0-3: 1;
 * the forcing term uses gamma_s and gamma_b as in eq. 14). */
enum { HSF_LB_BGK = 0, HSF_LB_MRT = 1 };

typedef struct {
    int iterations;              /* conjugate-gradient iterations               */
    int evaluations;             /* density-functional evaluations              */
    int restarts;                /* steepest-descent restarts                   */
    int converged;               /* residual <= tol                             */
    double residual;             /* max_I |phi_I[w] - phi_I| / |phi_I|          */
} hsf_invert_stats;

typedef struct hsf_ctx hsf_ctx;

/* Create a context for n_rep replicas described by reps[0..n_rep-1] on the
 * current HIP device.  The parameters are those of the model of section 2: the
 * chain architecture A_n B_m (+ monomeric solvent S) of eq. 2, the Flory-Huggins
 * parameters and Helfand compressibility of the free energy of eq. 1, the segment
 * length a of the Gaussian bond kernel discretised by the 27-point stencil
 * (text after eq. 17), the LB relaxation (eq. 10-15) and one time step shared by the
 * LB and convection-diffusion updates (text after eq. 17).  All replicas must share n_beads, types, has_solvent and
 * precision.  Densities start at zero, fields at zero, LB populations at rest
 * with density 1.  Returns HSF_EINVAL on inconsistent parameters, HSF_ENOMEM
 * when device memory is short.  Environment, read here: HSF_TILE=cx,cy,cz,k sets the
 * starting tiling; HSF_NO_GRAPHS=1 launches every kernel directly instead of replaying
 * captured sequences; HSF_POISON=1 fills every device buffer the context allocates (now
 * or later) with 0xff bytes, a NaN in FP32 and FP64, so that results that depend on memory
 * no kernel has written come out different (a checking aid; results are otherwise
 * unchanged). */
int hsf_create(const hsf_params *reps, int n_rep, hsf_ctx **out);

/* Free every device buffer of the context (waits for its stream). */
void hsf_destroy(hsf_ctx *ctx);

/* Message of the last failing call on this context (never NULL). */
const char *hsf_last_error(const hsf_ctx *ctx);

/* Order all further work of this context on the given hipStream_t (NULL: the
 * null stream).  The library never synchronises other streams. */
int hsf_set_stream(hsf_ctx *ctx, void *hip_stream);

/* Sizes and offsets, in elements, of the concatenated layouts above. */
long long hsf_total_sites(const hsf_ctx *ctx);
long long hsf_site_offset(const hsf_ctx *ctx, int rep);
long long hsf_field_offset(const hsf_ctx *ctx, int rep);
int hsf_num_species(const hsf_ctx *ctx);

/* Fields w_I = U_I / kT of all replicas (eq. 2). */
int hsf_set_fields(hsf_ctx *ctx, const double *w, int where);
int hsf_get_fields(hsf_ctx *ctx, double *w, int where);

/* Composition state phi_I = rho_I v0 of all replicas: the current densities of
 * the dynamics and the target of hsf_invert. */
int hsf_set_densities(hsf_ctx *ctx, const double *phi, int where);
int hsf_get_densities(hsf_ctx *ctx, double *phi, int where);

/* Density functional (eq. 2 via eq. 16-17): phi_out = phi[w] at the current
 * fields, with the copolymer amount phibar_p = <sum_polymer phi_I> and solvent
 * amount phibar_s = <phi_S> of the current densities (eq. 2 normalisation
 * n_p / Phi_p).  Q_out (n_rep values, may be NULL) receives the single-chain
 * partition function Q = V^-1 sum_r G_N(r) with G_0 = 1.  Does not change the
 * state.  phi_out uses the field layout. */
int hsf_evaluate(hsf_ctx *ctx, double *phi_out, double *Q_out, int where);

/* ---- allocation-free evaluation ----------------------------------------------
 * For callers that cannot allocate device memory (work recorded under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the density functional of
 * hsf_evaluate for ONE replica, without a context.  The call allocates and frees nothing:
 * its scratch (propagator store, field factors, partial sums, block tables, control
 * state) is a file-scope device array of HSF_STATIC_SCRATCH_BYTES that every GPU the
 * library runs on holds until the process ends.  It needs about
 * s (N + 4) V + 8 (N + 10) V / 256 bytes (s = 4 for FP32, 8 for FP64 propagators):
 * e.g. a 64^3 box with N <= 27 in FP64 or N <= 59 in FP32; larger problems return
 * HSF_EINVAL before anything is launched.
 *   p        one replica's parameters (box, chain, solvent, a or stencil, precision; the
 *            dynamics parameters are not used);
 *   w        device pointer, fields in the field layout [nsp][Lz][Ly][Lx], FP64;
 *   phi      device pointer, densities (same layout) whose amounts phibar_p and phibar_s
 *            normalise the result, as the current densities do in hsf_evaluate;
 *   phi_out  device pointer, phi[w] in the field layout;
 *   q_out    device pointer to one double: Q (NaN when it left the floating-point range);
 *   hip_stream  the hipStream_t the work is ordered on (NULL: the null stream).
 * The call only enqueues work and returns; results are ready when the stream is.  FP32
 * propagators run the evaluation twice, the first pass measuring the per-step
 * power-of-two scales the second uses.  Calls that overlap on one GPU share the array
 * and race; the caller orders them (one stream, or waits between streams).  Returns
 * HSF_OK, HSF_EINVAL (bad parameters, null pointers, box too large) or HSF_EHIP (a
 * launch failed). */
#define HSF_STATIC_SCRATCH_BYTES (64LL << 20)
int hsf_evaluate_static(const hsf_params *p, const double *w, const double *phi, double *phi_out, double *q_out,
                        void *hip_stream);

/* Observables of the current state (w, phi), n_rep values each (host memory, any
 * may be NULL):
 *   free_energy: the free-energy density v0 F / (kT V) of eq. 1 on the lattice,
 *     -n_p ln(V Q[w]) + ln n_p! - n_s ln sum_r exp(-w_S) + ln n_s!
 *     - sum_I sum_r phi_I w_I + 1/2 sum_IJ chi_IJ sum_r phi_I sigma[phi_J]
 *     + kappa/2 sum_r (sum_I phi_I - 1)^2, all over V, with n_p = phibar_p V / N,
 *     n_s = phibar_s V (phibar from phi) and sigma the linkage stencil; at
 *     self-consistent fields its derivative with respect to phi_I is the chemical
 *     potential of eq. 4;
 *   s_melt: sqrt(V^-1 sum_r sum_I (phi_I - <phi_I>)^2), the rms composition
 *     deviation (the melt's order parameter);
 *   s_sol: V^-1 sum_r |phi_A + phi_B - <phi_A> - <phi_B>|, the mean deviation of
 *     the copolymer total (the solution's order parameter).
 * Runs one density-functional evaluation (as hsf_evaluate) for Q and <exp(-w_S)>;
 * Q is computed with the context's propagator precision, the sums in FP64.
 * Does not change the state.  HSF_ENONFINITE when Q is not finite. */
int hsf_observables(hsf_ctx *ctx, double *free_energy, double *s_melt, double *s_sol);

/* Self-consistent fields for the current densities (section 2: Fletcher-Reeves
 * nonlinear conjugate gradients on the convex objective whose gradient is
 * phi^t - phi[w]).  The solvent field is set in closed form; polymer fields are
 * gauge-fixed to zero mean per species.  Stops when the residual
 * max_I |phi_I[w] - phi^t_I| / |phi^t_I| <= tol or after max_iter iterations.
 * stats (n_rep entries, may be NULL) receives per-replica counts.  Returns
 * HSF_ENOCONV when a replica stopped at max_iter (its iterate is kept). */
int hsf_invert(hsf_ctx *ctx, double tol, int max_iter, int warm, hsf_invert_stats *stats);

/* Chemical potentials (eq. 4) and force density (eq. 8) from the current
 * densities and fields.  mu: field layout; force: per replica [3][V] in LB
 * units, f = -dt^2 sum_I phi_I grad mu_I (central differences).  Either may
 * be NULL. */
int hsf_mu_force(hsf_ctx *ctx, double *mu, double *force, int where);

/* LB populations of all replicas, per replica [19][V], FP64 at this boundary.  With
 * FP32 storage (HSF_FP32 contexts) hsf_set_lb rounds each deviation n_i - w_i to FP32
 * (and allocates a staging buffer of 19 T doubles at the first call with host memory). */
int hsf_set_lb(hsf_ctx *ctx, const double *n, int where);
int hsf_get_lb(hsf_ctx *ctx, double *n, int where);

/* n_steps LB steps (eq. 10: collide, then stream) with a constant force
 * density (per replica [3][V], NULL for none).  rho/u of the last step's
 * pre-collision moments (eq. 9) are kept and returned by hsf_get_flow. */
int hsf_lb_advance(hsf_ctx *ctx, int n_steps, const double *force, int where);

/* Moments of the last LB step: rho per replica [V], u per replica [3][V]
 * (u includes the half-force shift of eq. 9).  Either may be NULL. */
int hsf_get_flow(hsf_ctx *ctx, double *rho, double *u, int where);

/* One conservative convection-diffusion update (eq. 3, explicit diffusive
 * flux, two-step Lax-Wendroff convective flux) of the current densities with
 * the given chemical potentials (field layout) and velocity (per replica
 * [3][V], NULL for none). */
int hsf_cd_advance(hsf_ctx *ctx, const double *mu, const double *u, int where);

/* Coupled steps (section 2, text after eq. 17: LB steps alternate with steps of the
 * convection-diffusion equation (3) at the same time step, and every such step first
 * determines the fields self-consistently by Fletcher-Reeves).  For each step: invert
 * (warm start of hsf_set_warm), then mu and force (eq. 4, 8), then (hydro on) one LB
 * step giving u (eq. 9-10), then the convection-diffusion update (eq. 3).  stats
 * (n_rep entries, may be NULL) receives the last step's inversion counts; total_evals
 * (may be NULL) the number of density-functional evaluations over all steps and
 * replicas.  Errors: HSF_ENOCONV when an inversion stops at max_iter (its iterate is
 * kept as the fields; densities and LB state are those of the step's start);
 * HSF_ENONFINITE when the inversion, an LB moment or an updated density is not finite
 * in some replica: the whole context is left as at the start of that step (fields,
 * densities, LB populations, scales, warm-start history, noise step word; the moments
 * read by hsf_get_flow are those of the failed step), the steps before it are kept. */
int hsf_step(hsf_ctx *ctx, int n_steps, double tol, int max_iter, hsf_invert_stats *stats,
             long long *total_evals);

/* Checkpoint of the state a continuation reads (section 3.2 continues runs from saved
 * states of earlier ones, e.g. switching the flow on in a state of a diffusion-only run,
 * Fig. 5-6): densities, fields, LB populations, the
 * replicas' inversion control state (with the per-step power-of-two scales of the FP32
 * propagators), the warm-start history, the noise step word and the propagator tiling.
 * hsf_get_state writes hsf_state_size(ctx) bytes into buf (host memory, size bytes);
 * hsf_set_state restores them into a context created with the same parameters, after
 * which further steps reproduce the checkpointed run bit for bit (given the same
 * solver, warm start, integrator and noise settings, which are configuration, not
 * state).  HSF_EINVAL for a short buffer, a buffer not written by hsf_get_state, or a
 * context of different replicas, species, chain, precision or size.  Both wait for the
 * context's stream. */
long long hsf_state_size(const hsf_ctx *ctx);
int hsf_get_state(hsf_ctx *ctx, void *buf, long long size);
int hsf_set_state(hsf_ctx *ctx, const void *buf, long long size);

/* Integrator of the convection-diffusion update of hsf_step (section 2).
 * HSF_CD_EXPLICIT (default): the explicit conservative step of hsf_cd_advance.
 * HSF_CD_CRANK_NICOLSON: the diffusive part implicit (Crank-Nicolson), convection by
 * the explicit two-step Lax-Wendroff flux and the noise of the step explicit:
 *   phi^{n+1} = phi^n + dt/2 [B(phi^n, mu^n) + B(phi^{n+1}, mu^{n+1})] - div J^C(phi^n, u^n) + xi^n,
 * B(phi, mu) = div(phi grad mu) with the face fluxes of the explicit step and
 * mu^{n+1} = mu[phi^{n+1}] (eq. 4 at the self-consistent fields of phi^{n+1}).  The
 * unknowns are those fields: phi^{n+1} = phi[w] with
 *   F(w) = phi[w] - dt/2 B(phi[w], mu(phi[w], w)) - rhs = 0,
 * solved for all replicas jointly by Newton's method with GMRES(krylov_dim) on
 * forward-difference Jacobian products (one density-functional evaluation each),
 * Krylov tolerance 1e-3 relative, corrections halved while they do not reduce ||F||,
 * until rms(F) <= tol or max_newton iterations (then hsf_step returns HSF_ENOCONV and
 * keeps the last iterate).  Newton starts from w^n.  After the step the densities are
 * phi[w^{n+1}] and the fields w^{n+1}, so the next step's inversion starts converged
 * (with Crank-Nicolson it always starts from the current fields).  The forward-difference
 * step is sqrt(2^-52) (1 + ||w||) with FP64 propagators; with FP32 propagators it is
 * 1e-4 (1 + ||w||), so that the evaluation's rounding stays small against the difference,
 * and the residual stalls at a few 1e-6 (the FP32 evaluation error carried through the
 * compressibility and the diffusive stencil): tol >= 1e-5 there.
 * HSF_EINVAL for tol <= 0 (or below 1e-5 with FP32 propagators), max_newton < 1 or
 * krylov_dim outside [2, 64].  Device memory: (krylov_dim + 6) nsp T doubles, allocated
 * at the first call. */
enum { HSF_CD_EXPLICIT = 0, HSF_CD_CRANK_NICOLSON = 1 };
int hsf_set_integrator(hsf_ctx *ctx, int scheme, double tol, int max_newton, int krylov_dim);

typedef struct {
    int newton;                  /* Newton iterations of the last Crank-Nicolson solve   */
    int krylov;                  /* Jacobian products (GMRES iterations), all Newton steps */
    long long evaluations;       /* density-functional evaluations, all replicas          */
    double residual;             /* final rms of F                                        */
    int converged;               /* residual <= tol                                       */
} hsf_cn_stats;
int hsf_get_cn_stats(const hsf_ctx *ctx, hsf_cn_stats *stats);

/* Thermal noise (off by default).  flags: HSF_NOISE_CD adds the composition noise
 * xi_I of eq. 5 to every convection-diffusion update, HSF_NOISE_LB the mode noise
 * phi_k r_k of eq. 13 to every LB collision; omega > 0 is the noise scaling parameter
 * Omega = h^3 / v0 (sec. 3).  In lattice units (h = 1, M = kT = 1 for eq. 3):
 *   LB: mode k >= 4 of the Table 1 basis gets sqrt(rho kT_LB b_k (1 - gamma_k^2) / c_s^2)
 *       r_k, kT_LB = dt^2 / Omega (the unit map of the force density), gamma_k of the
 *       collision (BGK: 1 - 1/tau for every non-conserved mode); mass and momentum are
 *       untouched;
 *   CD: each bond between r and r + e_a carries an extra flux
 *       sqrt(2 dt max((phi_I(r) + phi_I(r + e_a)) / 2, 0) / Omega) g, whose divergence
 *       has the covariance (2 dt / Omega)(-div phi_I grad) of eq. 5 over a step and
 *       conserves each species exactly.
 * Normal numbers: Philox4x64-10 (Salmon et al., SC11) of counter (site, step, purpose, 0)
 * under key (seed, replica index), two Box-Muller pairs per counter (radius from
 * ((x >> 11) + 1) 2^-53, angle 2 pi (x >> 11) 2^-53); purposes 0-3 the LB modes 4-18
 * (mode k takes number k - 4), 4 + I the bonds (x, y, z) of species I, a bond's numbers
 * being those of its lower site.  `step` is the step word of the next draw; every LB
 * step of hsf_lb_advance, every hsf_cd_advance and every coupled step of hsf_step
 * (both noises of it) uses the current value and then advances it by one, while noise
 * is on.  Waits for the context's stream.  HSF_EINVAL for unknown flags or a
 * non-positive Omega with noise on; flags = 0 switches noise off. */
enum { HSF_NOISE_CD = 1, HSF_NOISE_LB = 2 };
int hsf_set_noise(hsf_ctx *ctx, int flags, double omega, unsigned long long seed, unsigned long long step);
/* The step word of the next noise draw (to resume a run with the same numbers). */
int hsf_get_noise_step(const hsf_ctx *ctx, unsigned long long *step);

/* Switch convection by the LB flow on or off for every replica (the LB state
 * is kept while off).  Off is the diffusion-only model of section 3.1 (eq. 3 with
 * u = 0); section 3.2 turns the flow on, or off, part way through a run (Fig. 5-7). */
int hsf_set_hydro(hsf_ctx *ctx, int on);

/* Inversion variant.  0 (default): plain Fletcher-Reeves on the gradient
 * g = phi^t - phi[w].  HSF_SOLVER_PRECOND: the steepest-descent vector is
 * z = g / phi^t (diagonal preconditioning by the target densities), with
 * beta = (g_new.z_new)/(g_old.z_old); same line search and stopping test.
 * HSF_SOLVER_REFINE (FP32 contexts; no effect in FP64 ones): the FP32 propagators'
 * rounding bounds the residual an inversion can reach (1e-7 to 3e-6, by box and
 * composition); with this flag an inversion asked for a residual below 1e-5 iterates with
 * FP32 evaluations down to 1e-5 and then with FP64 evaluations (the same iteration,
 * restarted along the steepest descent direction) down to tol, each phase with at most
 * max_iter iterations; the
 * statistics add up both phases.  The first call that sets it allocates the FP64
 * propagators (8 (N + 6) bytes per site; HSF_ENOMEM if short); HSF_EINVAL if the tiling
 * in use does not fit the LDS in FP64, and while it is on hsf_set_tile and hsf_autotune
 * only take tilings that do. */
enum { HSF_SOLVER_PRECOND = 1, HSF_SOLVER_REFINE = 2 };
int hsf_set_solver(hsf_ctx *ctx, int flags);

/* Work done by inversions since creation or the last reset: the number of
 * density-functional evaluations over all replicas, and the sum over replicas of
 * evaluations times sites (each evaluation performs 2 N site-bead updates per
 * site).  reset != 0 clears both counters after reading. */
int hsf_get_work(hsf_ctx *ctx, long long *evals, double *site_evals, int reset);

/* Propagator tiling (the temporally blocked sweeps): cfg = {cx, cy, cz, k}, a
 * core tile of cx*cy*cz sites per workgroup advanced k contour steps per launch;
 * k = 0: one step per launch, read through the caches; k = -1: as k = 0, but each
 * launch takes a forward and a backward step together (N + 1 launches per
 * evaluation instead of 2 N, densities bit for bit those of k = 0).
 * hsf_set_tile accepts only the configurations compiled into the library
 * (HSF_EINVAL otherwise); results do not depend on the choice beyond rounding.
 * hsf_autotune times one density-functional evaluation `reps` times with every
 * configuration that fits the device's LDS and keeps the fastest (best_ms, may be
 * NULL, receives its time).  It leaves densities, fields and LB state unchanged. */
int hsf_set_tile(hsf_ctx *ctx, const int cfg[4]);
int hsf_get_tile(const hsf_ctx *ctx, int cfg[4]);
int hsf_autotune(hsf_ctx *ctx, int reps, double *best_ms);

/* Schedule of the paired sweeps (tilings with k = -1) for chains of n_beads >= 2 beads,
 * the order in which eq. 17's forward steps and eq. 16-17's backward steps are launched:
 * launch j (1..n_beads) takes forward step out[0] = j and backward step out[1] (0: none),
 * with the flags out[2..7] = f_late (the forward step finds sigma[G+_{s+1}] in the store
 * slot of its bead and stores the density term), f_from_pp (it reads G_{s-1} from its
 * ping-pong pair), f_to_pp (it also writes G_s there), g_late (the backward step finds G_s
 * in the slot and stores the term; else it stores sigma[G+_{s+1}]), g_exp (it forms its
 * field factor from the fields) and g_from_e (backward step N - 1 of an even chain of at
 * least 4 beads, whose backward step N has no launch: its stencil reads G+_N as bead N's
 * stored field factor times csum and the step-N scale).  Backward step 1 follows alone.
 * Host computation only (the evaluation uses the same function); HSF_EINVAL for n_beads
 * outside 2..64 or launch outside 1..n_beads. */
int hsf_paired_schedule(int n_beads, int launch, int out[8]);

/* Warm start used by hsf_step's inversions (default HSF_WARM_CURRENT). */
int hsf_set_warm(hsf_ctx *ctx, int warm);

/* ---- learned warm start -------------------------------------------------------
 * A U-Net of D = 1..4 levels on the periodic lattice (3x3x3 convolutions, SiLU,
 * 2x2x2 average pooling, nearest upsampling, additive skips) mapping in_ch input
 * channels to out_ch output channels on the same L^3 box.  widths[0..D-1] (each
 * 1..32) are the level widths and widths[D..3] are zero.  Convolutions run on the
 * BF16 matrix cores with FP32 accumulation; master weights and Adam moments are
 * FP32.  Tensors at this boundary are FP32 [batch][channel][Lz][Ly][Lx] on cubic
 * periodic boxes with L a multiple of 2^(D-1).  The parameter vector holds, for the
 * 4 D - 1 convolutions in order (per encoder level its two, per decoder level from
 * the coarsest its two, then the output convolution), W[co][ci][27] with
 * k = 9 (dz+1) + 3 (dy+1) + (dx+1), then b[co].  Device buffers are owned by the
 * network; pointers passed in are borrowed for the call.  Errors: HSF_EINVAL for bad
 * sizes or pointers, HSF_ENOMEM, HSF_EHIP (hsf_net_last_error has the message).
 * This is a build addition; the inversion from its prediction is the same
 * Fletcher-Reeves iteration to the same residual. */
typedef struct hsf_net hsf_net;
int hsf_net_create(int in_ch, int out_ch, const int widths[4], unsigned long long seed, hsf_net **out);
void hsf_net_destroy(hsf_net *net);
const char *hsf_net_last_error(const hsf_net *net);
int hsf_net_set_stream(hsf_net *net, void *hip_stream);
long long hsf_net_num_params(const hsf_net *net);
int hsf_net_set_params(hsf_net *net, const float *params, int where);
/* Input normalisation applied inside every forward pass: x_c = (in_c - shift[c]) *
 * scale[c] (host arrays of in_ch values; default shift 0, scale 1). */
int hsf_net_set_input_norm(hsf_net *net, const float *shift, const float *scale);
/* Output scale applied at the end of every forward pass: out_c *= scale[c] (host array
 * of out_ch values; default 1).  A network is trained on targets divided by the scale
 * with the scale at 1 (hsf_net_loss_grad and hsf_net_train_step refuse, HSF_EINVAL,
 * while a scale other than 1 is set) and deployed with it. */
int hsf_net_set_output_scale(hsf_net *net, const float *scale);
int hsf_net_get_params(hsf_net *net, float *params, int where);
/* out = net(in) for `batch` samples */
int hsf_net_forward(hsf_net *net, const float *in, float *out, int batch, int L, int where);
/* mean square error over batch, channels and sites, and its gradient with respect
 * to the parameters (grad may be NULL) */
int hsf_net_loss_grad(hsf_net *net, const float *in, const float *target, int batch, int L, double *loss,
                      float *grad, int where);
/* one Adam step (beta 0.9, 0.999, eps 1e-8) on the mean square error */
int hsf_net_train_step(hsf_net *net, const float *in, const float *target, int batch, int L, float lr,
                       double *loss, int where);
/* Training data of the warm starts, assembled on the device (the network's stream), for
 * one replica from up to three states of an inversion trajectory: the target densities
 * and converged fields phi, w of a step, phi_n, w_n of the step before and phi_p, w_p of
 * the one before that (device pointers, field layout [nsp][V], FP64).  Mode 0 (the direct
 * map of HSF_WARM_NET): x (device, FP32 [nsp][V]) receives phi and y (device, FP32 [2][V])
 * the polymer fields w; phi_n, w_n, phi_p, w_p may be NULL.  Modes 1 and 2: x (FP32
 * [2 nsp][V]) receives the input HSF_WARM_NET_DELTA (mode 1) or HSF_WARM_NET_EXTRAP
 * (mode 2) feeds the network, (phi_n, delta phi / r), and y (FP32 [2][V]) the matching
 * target delta w / r of the polymer fields, with delta the first (mode 1: phi - phi_n) or
 * second (mode 2: phi - 2 phi_n + phi_p) difference and r the rms of delta phi over
 * species and sites; phi_p, w_p may be NULL in mode 1. */
int hsf_net_make_sample(hsf_net *net, const double *phi, const double *phi_n, const double *phi_p, const double *w,
                        const double *w_n, const double *w_p, int nsp, long long V, int mode, float *x, float *y);
/* x_c = (x_c - shift[c]) * scale[c] for each channel c of x (device, FP32
 * [batch][channels][V]); shift and scale are host arrays of `channels` values (used to
 * bring training targets to unit scale per channel).  Waits for the network's stream. */
int hsf_net_affine(hsf_net *net, float *x, int batch, int channels, long long V, const float *shift,
                   const float *scale);
/* Mean and root mean square of each of `channels` channels of x (device, FP32
 * [batch][channels][V]) over samples and sites, into the host arrays mean[] and rms[]
 * (for the input normalisation and output scale of a training set).  Waits for the
 * network's stream. */
int hsf_net_channel_moments(hsf_net *net, const float *x, int batch, int channels, long long V, double *mean,
                            double *rms);
/* Attach a network to a context for the NET warm starts (in_ch = nsp for
 * HSF_WARM_NET, 2 nsp for HSF_WARM_NET_DELTA and HSF_WARM_NET_EXTRAP; out_ch = 2;
 * replicas with equal boxes are predicted in one batch);
 * the context does not own it.  NULL detaches.  The inputs the network sees for
 * one replica are FP32 [channel][V]: HSF_WARM_NET the target densities; the delta
 * modes phi^n (nsp channels) followed by the density difference divided by r. */
int hsf_attach_net(hsf_ctx *ctx, hsf_net *net);
/* Use the network in HSF_WARM_NET_DELTA / HSF_WARM_NET_EXTRAP only when the previous
 * inversion of some replica took at least min_iters iterations; otherwise take the
 * plain counterpart (the held fields, or the extrapolation).  0 (the default) always
 * uses the network.  HSF_EINVAL for a negative value. */
int hsf_set_net_gate(hsf_ctx *ctx, int min_iters);

/* Kernel families timed by hsf_set_timing. */
enum {
    HSF_K_PREP = 0,   /* field preparation + first forward step          */
    HSF_K_FWD = 1,    /* forward propagator step                         */
    HSF_K_BWD = 2,    /* backward propagator step + density accumulation */
    HSF_K_LB = 3,     /* fused LB collide-and-stream                     */
    HSF_K_CD = 4,     /* convection-diffusion update                     */
    HSF_K_PAIR = 5,   /* paired launch: one forward and one backward step */
    HSF_K_COUNT = 6
};

/* Measurement aid: when on, every launch of the kernel families above is
 * bracketed by HIP events recorded on the context's stream.  hsf_get_timing
 * waits for the stream and returns, per family, the summed event-to-event time
 * in milliseconds (total_ms[HSF_K_COUNT]) and the number of launches
 * (count[HSF_K_COUNT]) since the previous read, then clears them. */
int hsf_set_timing(hsf_ctx *ctx, int on);
int hsf_get_timing(hsf_ctx *ctx, double *total_ms, long long *count);

/* Step log: one record per replica and successful coupled step (hsf_step), kept while
 * the log is on.  It follows a run the way the paper follows its simulations in time
 * (section 3: morphologies and order parameters against the time step): the step's
 * inversion (iterations, evaluations, final residual, ln Q at the converged fields), the
 * amount of each species and the largest flow speed after the step, and the wall time
 * of the step's two phases (inversion; LB and convection-diffusion), from HIP events
 * on the context's stream and shared by the replicas of the step.  Recording costs one
 * pass over the densities and velocities and one small copy per step.  Failed steps are
 * not recorded. */
typedef struct {
    long long step;       /* successful coupled steps of this context since hsf_create, this one included */
    int replica;
    int iterations, evaluations, converged;
    double residual;
    double ln_q;
    double amount[3];     /* site sums of phi_A, phi_B, phi_S (phi_S 0 for melts) after the step */
    double max_u;         /* largest |u| of the step's LB velocity (0 with the flow off) */
    double ms_inversion;
    double ms_dynamics;
} hsf_step_record;
/* on = 1 starts keeping records (at most 1 << 20; beyond that the oldest are dropped),
 * on = 0 stops and drops the unread ones.  HSF_EINVAL for a null context. */
int hsf_set_step_log(hsf_ctx *ctx, int on);
/* Moves up to max_records of the oldest unread records into out (host array) and sets
 * *n_read to their number.  HSF_EINVAL for a null context, out or n_read, or a negative
 * max_records. */
int hsf_read_step_log(hsf_ctx *ctx, hsf_step_record *out, int max_records, int *n_read);

#ifdef __cplusplus
}
#endif

#endif /* HSF_H */
