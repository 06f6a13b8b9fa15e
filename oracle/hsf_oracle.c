/*
 * hsf_oracle.c -- plain FP64 CPU oracle of the hybrid lattice-Boltzmann /
 * dynamic self-consistent-field method of Zhang, Sevink and Schmid,
 * "Hybrid Lattice Boltzmann/Dynamic Self-Consistent Field Simulations of
 * Microphase Separation and Vesicle Formation in Block Copolymer Systems"
 * (arXiv:1204.2088).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * compared against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant generator with the HIP library; every formula below is written out
 * directly from the paper in plain loops, slow on purpose, in double precision.
 *
 * Where the paper is silent or garbled, the reading taken is named in the
 * comment of the function that uses it (readings are also listed in the
 * design notes of the repository).
 *
 * Every function here is pinned by tests against values fixed by the paper or
 * by mathematics (closed forms, brute force, Fourier linear response,
 * conservation laws, Taylor-Green decay).  No function is "parity unpinned".
 *
 * Timing only: built with -fopenmp (the benchmark's all-core CPU baseline) the
 * site loops marked "omp" run over z-planes (or sites) in parallel.  Each
 * iteration writes its own outputs and every sum stays in a serial loop, so
 * the results are bit for bit those of the plain build.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_BEADS 64

/* System description.  Species index: 0 = A, 1 = B, 2 = S (solvent). */
typedef struct {
    int Lx, Ly, Lz;              /* periodic box, lattice spacing h = 1       */
    int N;                       /* beads per copolymer chain                 */
    int types[ORC_MAX_BEADS];    /* species of bead s = 1..N stored at [s-1]  */
    int n_poly;                  /* polymer species (2: A and B)              */
    int has_solvent;             /* 1: monomeric solvent S is species 2       */
    double c[4];                 /* stencil weights: centre, face, edge, corner */
    double chi[3][3];            /* Flory-Huggins chi_IJ (symmetric)          */
    double kappa;                /* Helfand compressibility kappa_H v0 / kT   */
    double dt;                   /* time step in diffusive units              */
    double tau;                  /* BGK relaxation time                       */
    double gamma_b, gamma_s, gamma_ghost; /* MRT relaxation parameters        */
    int lb_mode;                 /* 0: BGK + Guo forcing, 1: MRT (Table 1)    */
    int hydro;                   /* 1: convection by the LB velocity          */
    int precond;                 /* 1: inversion preconditioned by diag(phi^t) */
    int noise;                   /* bit 0: composition noise (eq. 5), bit 1: LB mode noise (eq. 13) */
    double omega;                /* noise scaling parameter Omega = h^3 / v0 (sec. 3) */
    unsigned long long seed;     /* generator key, first word */
    unsigned long long rep;      /* generator key, second word (replica index) */
    unsigned long long step;     /* time-step word of the generator counter */
} orc_sys;

typedef struct {
    int iterations;
    int evaluations;
    int restarts;
    double residual;
    int converged;
} orc_invert_stats;

static long vol(const orc_sys *s) { return (long)s->Lx * s->Ly * s->Lz; }
static int nsp(const orc_sys *s) { return s->n_poly + (s->has_solvent ? 1 : 0); }

static int wrap(int i, int L) { return ((i % L) + L) % L; }

static long site(const orc_sys *s, int x, int y, int z)
{
    return (long)wrap(x, s->Lx) + (long)s->Lx * ((long)wrap(y, s->Ly) + (long)s->Ly * wrap(z, s->Lz));
}

/*
 * Stencil weights from the statistical segment length a (paper section 2:
 * a = 1.1543 h; the 27-point scheme itself is only cited, not printed).
 * Reading: tensor product of the 1-D kernel [alpha, 1-2 alpha, alpha] with
 * alpha = a^2/6, which keeps the normalisation and the per-axis bond variance
 * a^2/3 of the continuum Gaussian bond of the Edwards Hamiltonian.
 */
void orc_stencil_weights(double a, double c[4])
{
    double al = a * a / 6.0;
    double ce = 1.0 - 2.0 * al;
    c[0] = ce * ce * ce;
    c[1] = al * ce * ce;
    c[2] = al * al * ce;
    c[3] = al * al * al;
}

/*
 * Linkage operator sigma (eq. 17, the Gaussian convolution) on the lattice:
 * a 27-point stencil whose weight depends only on how many of the three
 * components of the offset are non-zero.  Periodic boundaries.
 */
void orc_sigma(const orc_sys *s, const double *f, double *out)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->Lz; ++z)
        for (int y = 0; y < s->Ly; ++y)
            for (int x = 0; x < s->Lx; ++x) {
                double acc = 0.0;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int k = (dx != 0) + (dy != 0) + (dz != 0);
                            acc += s->c[k] * f[site(s, x + dx, y + dy, z + dz)];
                        }
                out[site(s, x, y, z)] = acc;
            }
}

/*
 * Density functional (eq. 2 through the propagator form eq. 16-17).
 *   G_0 = 1,        G_s  = exp(-w_{t_s}) sigma[G_{s-1}],   s = 1..N
 *   G+_{N+1} = 1,   G+_s = exp(-w_{t_s}) sigma[G+_{s+1}],  s = N..1
 *   Q   = V^-1 sum_r G_N(r)
 *   phi_I(r) = phibar_p / (N Q) * sum_{s: t_s = I} G_s(r) sigma[G+_{s+1}](r)
 *   phi_S(r) = phibar_s exp(-w_S(r)) / <exp(-w_S)>        (eq. 2, solvent)
 * The proportionality of eq. 16 is fixed by the normalisation n_p/Phi_p of
 * eq. 2, with the copolymer amount phibar_p taken as an input (reading).
 * Qs[s-1] (optional) receives V^-1 sum_r G_s sigma[G+_{s+1}], which equals Q
 * for every s.
 * w and phi are [species][V].  Returns 0, or -1 on allocation failure.
 */
int orc_evaluate(const orc_sys *s, const double *w, double phibar_p, double phibar_s,
                 double *phi, double *Q, double *Qs)
{
    long V = vol(s);
    int N = s->N;
    double *G = malloc(sizeof(double) * V * (N + 1));
    double *E = malloc(sizeof(double) * V * s->n_poly);
    double *Gp = malloc(sizeof(double) * V);
    double *S = malloc(sizeof(double) * V);
    double *acc = calloc((size_t)V * s->n_poly, sizeof(double));
    if (!G || !E || !Gp || !S || !acc) {
        free(G); free(E); free(Gp); free(S); free(acc);
        return -1;
    }
    for (int I = 0; I < s->n_poly; ++I)
#pragma omp parallel for schedule(static)
        for (long r = 0; r < V; ++r)
            E[I * V + r] = exp(-w[I * V + r]);

    for (long r = 0; r < V; ++r) G[r] = 1.0;
    for (int k = 1; k <= N; ++k) {
        const double *Ek = E + (long)s->types[k - 1] * V;
        orc_sigma(s, G + (long)(k - 1) * V, S);
#pragma omp parallel for schedule(static)
        for (long r = 0; r < V; ++r) G[(long)k * V + r] = Ek[r] * S[r];
    }
    double q = 0.0;
    for (long r = 0; r < V; ++r) q += G[(long)N * V + r];
    q /= (double)V;

    for (long r = 0; r < V; ++r) Gp[r] = 1.0;
    for (int k = N; k >= 1; --k) {
        int I = s->types[k - 1];
        orc_sigma(s, Gp, S);
#pragma omp parallel for schedule(static)
        for (long r = 0; r < V; ++r) acc[I * V + r] += G[(long)k * V + r] * S[r];
        if (Qs) {
            double qs = 0.0;
            for (long r = 0; r < V; ++r) qs += G[(long)k * V + r] * S[r];
            Qs[k - 1] = qs / (double)V;
        }
#pragma omp parallel for schedule(static)
        for (long r = 0; r < V; ++r) Gp[r] = E[I * V + r] * S[r];
    }
    double pref = phibar_p / ((double)N * q);
    for (int I = 0; I < s->n_poly; ++I)
        for (long r = 0; r < V; ++r) phi[I * V + r] = pref * acc[I * V + r];

    if (s->has_solvent) {
        const double *wS = w + (long)s->n_poly * V;
        double m = 0.0;
        for (long r = 0; r < V; ++r) m += exp(-wS[r]);
        m /= (double)V;
        for (long r = 0; r < V; ++r) phi[(long)s->n_poly * V + r] = phibar_s * exp(-wS[r]) / m;
    }
    if (Q) *Q = q;
    free(G); free(E); free(Gp); free(S); free(acc);
    return 0;
}

/* ln Q[w] for the objective used by the inversion (diagnostic / FD checks). */
double orc_log_q(const orc_sys *s, const double *w)
{
    long V = vol(s);
    double *phi = malloc(sizeof(double) * V * nsp(s));
    double q = NAN;
    if (phi && orc_evaluate(s, w, 1.0, 1.0, phi, &q, NULL) != 0) q = NAN;
    free(phi);
    return log(q);
}

static double dot(const double *a, const double *b, long n)
{
    double acc = 0.0;
    for (long i = 0; i < n; ++i) acc += a[i] * b[i];
    return acc;
}

/* max over polymer species of ||phi_I - phi^t_I|| / ||phi^t_I|| with g = phi^t - phi */
static double residual(const orc_sys *s, const double *g, const double *phit)
{
    long V = vol(s);
    double res = 0.0;
    for (int I = 0; I < s->n_poly; ++I) {
        double num = dot(g + I * V, g + I * V, V);
        double den = dot(phit + I * V, phit + I * V, V);
        double r = sqrt(num / den);
        if (!(r <= res)) res = r; /* NaN propagates */
    }
    return res;
}

/*
 * Self-consistent determination of the fields from the densities (paper
 * section 2: every convection-diffusion step determines U_I self-consistently
 * with the Fletcher-Reeves nonlinear conjugate gradient method).
 *
 * Reading of the unspecified details: the fields minimise the convex
 *   Phi(w) = (phibar_p V / N) ln Q[w] + phibar_s V ln<exp(-w_S)> + sum_I sum_r phi^t_I w_I
 * whose gradient is phi^t - phi[w], so phi[w] = phi^t at the minimum.
 *   - the solvent field is set in closed form, w_S = -ln(phi^t_S / phibar_s);
 *   - polymer fields are gauge-fixed to zero mean per species at the start
 *     (densities do not change under a constant shift per species);
 *   - line search: secant on h(alpha) = d . grad Phi(w + alpha d) starting at
 *     alpha_0 = -(d.g) / sum d^2 phi^t (diagonal Hessian estimate), accepting
 *     when |h| <= 0.1 |h(0)| or after 3 trial points; a trial is also
 *     accepted when the secant slope is not positive or the next alpha is not
 *     positive; extrapolation is capped at 8x the current alpha;
 *   - Fletcher-Reeves beta = |g_new|^2 / |g_old|^2, restart (d = -g) every 50
 *     iterations and whenever d.g >= 0;
 *   - optional diagonal preconditioning (precond = 1): the steepest-descent
 *     vector is z = g / phi^t instead of g, so d = -z + beta d with
 *     beta = (g_new.z_new) / (g_old.z_old) and restarts set d = -z;
 *   - stop when max_I |phi_I - phi^t_I| / |phi^t_I| <= tol.
 * With fixed_iters > 0 exactly that many iterations are taken whatever the
 * residual ("mirror" mode, to follow another implementation's trajectory).
 *
 * phit and w are [species][V]; w holds the starting guess on entry and the
 * result on exit.  Returns 0 when converged (or fixed_iters done), 1 when
 * max_iter was reached, -1 on allocation failure.
 */
int orc_invert(const orc_sys *s, const double *phit, double *w, double tol, int max_iter,
               int fixed_iters, orc_invert_stats *st)
{
    long V = vol(s);
    int ns = nsp(s);
    long n = (long)s->n_poly * V;
    double phibar_p = 0.0, phibar_s = 0.0;
    for (int I = 0; I < s->n_poly; ++I)
        for (long r = 0; r < V; ++r) phibar_p += phit[I * V + r];
    phibar_p /= (double)V;
    if (s->has_solvent) {
        for (long r = 0; r < V; ++r) phibar_s += phit[(long)s->n_poly * V + r];
        phibar_s /= (double)V;
        for (long r = 0; r < V; ++r)
            w[(long)s->n_poly * V + r] = -log(phit[(long)s->n_poly * V + r] / phibar_s);
    }
    for (int I = 0; I < s->n_poly; ++I) {
        double m = 0.0;
        for (long r = 0; r < V; ++r) m += w[I * V + r];
        m /= (double)V;
        for (long r = 0; r < V; ++r) w[I * V + r] -= m;
    }

    double *phi = malloc(sizeof(double) * V * ns);
    double *g = malloc(sizeof(double) * n);
    double *d = malloc(sizeof(double) * n);
    double *wt = malloc(sizeof(double) * V * ns);
    double *gt = malloc(sizeof(double) * n);
    if (!phi || !g || !d || !wt || !gt) {
        free(phi); free(g); free(d); free(wt); free(gt);
        return -1;
    }
    orc_invert_stats loc = {0, 0, 0, 0.0, 0};

    orc_evaluate(s, w, phibar_p, phibar_s, phi, NULL, NULL);
    loc.evaluations = 1;
    for (long i = 0; i < n; ++i) g[i] = phit[i] - phi[i];
    loc.residual = residual(s, g, phit);
    int status = 1;
    if (fixed_iters <= 0 && loc.residual <= tol) status = 0;

    if (status != 0) {
        /* z = M^-1 g with M = diag(phi^t) when preconditioned, else z = g */
#define ZI(i) (s->precond ? g[i] / phit[i] : g[i])
        for (long i = 0; i < n; ++i) d[i] = -ZI(i);
        double gg = 0.0;
        for (long i = 0; i < n; ++i) gg += g[i] * ZI(i);
        int limit = fixed_iters > 0 ? fixed_iters : max_iter;
        memcpy(wt, w, sizeof(double) * V * ns);
        for (int k = 1; k <= limit; ++k) {
            double h0 = dot(d, g, n);
            if (h0 >= 0.0) {
                for (long i = 0; i < n; ++i) d[i] = -ZI(i);
                h0 = -gg;
                loc.restarts++;
            }
            double dhd = 0.0;
            for (long i = 0; i < n; ++i) dhd += d[i] * d[i] * phit[i];
            double alpha = -h0 / dhd;
            double a_prev = 0.0, h_prev = h0;
            for (int t = 1; t <= 3; ++t) {
                for (long i = 0; i < n; ++i) wt[i] = w[i] + alpha * d[i];
                orc_evaluate(s, wt, phibar_p, phibar_s, phi, NULL, NULL);
                loc.evaluations++;
                for (long i = 0; i < n; ++i) gt[i] = phit[i] - phi[i];
                double h = dot(d, gt, n);
                if (fabs(h) <= 0.1 * fabs(h0) || t == 3) break;
                double slope = (h - h_prev) / (alpha - a_prev);
                if (!(slope > 0.0)) break;
                double a_new = alpha - h / slope;
                if (!(a_new > 0.0)) break;
                if (a_new > 8.0 * alpha) a_new = 8.0 * alpha;
                a_prev = alpha;
                h_prev = h;
                alpha = a_new;
            }
            memcpy(w, wt, sizeof(double) * n);
            memcpy(g, gt, sizeof(double) * n);
            loc.iterations = k;
            loc.residual = residual(s, g, phit);
            if (fixed_iters <= 0 && loc.residual <= tol) {
                status = 0;
                break;
            }
            double gg_new = 0.0;
            for (long i = 0; i < n; ++i) gg_new += g[i] * ZI(i);
            double beta = gg_new / gg;
            gg = gg_new;
            if (k % 50 == 0) {
                beta = 0.0;
                loc.restarts++;
            }
            for (long i = 0; i < n; ++i) d[i] = -ZI(i) + beta * d[i];
        }
#undef ZI
        if (fixed_iters > 0) status = 0;
    }
    loc.converged = (loc.residual <= tol);
    if (st) *st = loc;
    free(phi); free(g); free(d); free(wt); free(gt);
    return status;
}

/*
 * Intrinsic chemical potential (eq. 4) and thermodynamic volume force (eq. 8).
 *   mu_I = -w_I + sum_J chi_IJ sigma[phi_J] + kappa (sum_J phi_J - 1)
 * Readings: the Gaussian interaction kernel of eq. 1 has the same width a as
 * the bond kernel and is discretised with the same stencil; eps0_II = 0 so
 * that eps0_IJ v0 / kT = chi_IJ; the volume fraction phi_I = rho_I v0.
 * Force in lattice-Boltzmann units (h = lattice step = 1; bead mass
 * m0 = kT tau^2 / h^2; the LB step equals the diffusive step dt):
 *   f_alpha = -dt^2 sum_I phi_I (mu_I(r + e_alpha) - mu_I(r - e_alpha)) / 2
 * (central difference; the paper does not state the gradient discretisation).
 * phi, w, mu: [species][V]; f: [3][V].
 */
void orc_mu_force(const orc_sys *s, const double *phi, const double *w, double *mu, double *f)
{
    long V = vol(s);
    int ns = nsp(s);
    double *sp = malloc(sizeof(double) * V * ns);
    for (int J = 0; J < ns; ++J) orc_sigma(s, phi + (long)J * V, sp + (long)J * V);
    for (int I = 0; I < ns; ++I)
        for (long r = 0; r < V; ++r) {
            double tot = 0.0, inter = 0.0;
            for (int J = 0; J < ns; ++J) {
                tot += phi[(long)J * V + r];
                inter += s->chi[I][J] * sp[(long)J * V + r];
            }
            mu[(long)I * V + r] = -w[(long)I * V + r] + inter + s->kappa * (tot - 1.0);
        }
    free(sp);
    if (!f) return;
    for (int z = 0; z < s->Lz; ++z)
        for (int y = 0; y < s->Ly; ++y)
            for (int x = 0; x < s->Lx; ++x) {
                long r = site(s, x, y, z);
                double fx = 0.0, fy = 0.0, fz = 0.0;
                for (int I = 0; I < ns; ++I) {
                    const double *m = mu + (long)I * V;
                    double p = phi[(long)I * V + r];
                    fx += p * 0.5 * (m[site(s, x + 1, y, z)] - m[site(s, x - 1, y, z)]);
                    fy += p * 0.5 * (m[site(s, x, y + 1, z)] - m[site(s, x, y - 1, z)]);
                    fz += p * 0.5 * (m[site(s, x, y, z + 1)] - m[site(s, x, y, z - 1)]);
                }
                double k = -s->dt * s->dt;
                f[r] = k * fx;
                f[V + r] = k * fy;
                f[2 * V + r] = k * fz;
            }
}

/*
 * Free-energy density v0 F / (kT V) of eq. 1 on the lattice (v0 = 1, kT = 1,
 * integrals as site sums), at fields w and volume fractions phi:
 *   F = -n_p ln Phi_p - n_s ln Phi_s + ln n_p! + ln n_s!
 *       - sum_I sum_r phi_I w_I
 *       + 1/2 sum_IJ chi_IJ sum_r phi_I sigma[phi_J]
 *       + kappa/2 sum_r (sum_I phi_I - 1)^2
 * with Phi_p = sum_r G_N(r) = V Q[w] (the single-chain partition function of the
 * copolymer in the fields), Phi_s = sum_r exp(-w_S), n_p = phibar_p V / N chains
 * and n_s = phibar_s V solvent beads (phibar from the given phi), ln n! = lgamma(n + 1).
 * The interaction kernel is the linkage stencil with eps0_IJ = chi_IJ (the same
 * reading as the chemical potential of eq. 4, which is the derivative of this F).
 * Returns NAN on allocation failure.
 */
double orc_free_energy(const orc_sys *s, const double *w, const double *phi)
{
    long V = vol(s);
    int ns = nsp(s);
    double pbar_p = 0.0, pbar_s = 0.0;
    for (long r = 0; r < V; ++r) {
        for (int I = 0; I < s->n_poly; ++I) pbar_p += phi[(long)I * V + r];
        if (s->has_solvent) pbar_s += phi[(long)s->n_poly * V + r];
    }
    pbar_p /= (double)V;
    pbar_s /= (double)V;
    double *tmp = malloc(sizeof(double) * V * ns);
    double *sp = malloc(sizeof(double) * V * ns);
    if (!tmp || !sp) {
        free(tmp);
        free(sp);
        return NAN;
    }
    double q = NAN;
    if (orc_evaluate(s, w, pbar_p, pbar_s, tmp, &q, NULL) != 0) q = NAN;
    const double np = pbar_p * (double)V / (double)s->N, nsol = pbar_s * (double)V;
    double F = -np * log((double)V * q) + lgamma(np + 1.0);
    if (s->has_solvent) {
        double zs = 0.0;
        const double *wS = w + (long)s->n_poly * V;
        for (long r = 0; r < V; ++r) zs += exp(-wS[r]);
        F += -nsol * log(zs) + lgamma(nsol + 1.0);
    }
    for (int J = 0; J < ns; ++J) orc_sigma(s, phi + (long)J * V, sp + (long)J * V);
    double fw = 0.0, fi = 0.0, fk = 0.0;
    for (long r = 0; r < V; ++r) {
        double tot = 0.0;
        for (int I = 0; I < ns; ++I) {
            const double pI = phi[(long)I * V + r];
            tot += pI;
            fw += pI * w[(long)I * V + r];
            for (int J = 0; J < ns; ++J) fi += 0.5 * s->chi[I][J] * pI * sp[(long)J * V + r];
        }
        fk += 0.5 * s->kappa * (tot - 1.0) * (tot - 1.0);
    }
    F += -fw + fi + fk;
    free(tmp);
    free(sp);
    return F / (double)V;
}

/*
 * Order parameters of the composition phi [species][V] (phi^0_I: the spatial mean
 * of phi_I): the melt's S = sqrt(V^-1 sum_r sum_I (phi_I - phi^0_I)^2) and the
 * solution's S = V^-1 sum_r |phi_A + phi_B - phi^0_A - phi^0_B|.
 */
void orc_order_params(const orc_sys *s, const double *phi, double *s_melt, double *s_sol)
{
    long V = vol(s);
    int ns = nsp(s);
    double mean[3] = {0.0, 0.0, 0.0};
    for (int I = 0; I < ns; ++I) {
        for (long r = 0; r < V; ++r) mean[I] += phi[(long)I * V + r];
        mean[I] /= (double)V;
    }
    double sq = 0.0, ab = 0.0;
    for (long r = 0; r < V; ++r) {
        for (int I = 0; I < ns; ++I) {
            const double d = phi[(long)I * V + r] - mean[I];
            sq += d * d;
        }
        ab += fabs(phi[r] + phi[V + r] - mean[0] - mean[1]);
    }
    *s_melt = sqrt(sq / (double)V);
    *s_sol = ab / (double)V;
}

/*
 * Counter-based random numbers for the thermal noise: Philox4x64 with 10 rounds
 * (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC11).  A round multiplies counter words 0 and 2 by two fixed odd constants
 * (128-bit products), and forms the new words from the high halves xored with
 * words 1 / 3 and the round key, and the low halves; the key is advanced by two
 * Weyl increments between rounds.
 */
typedef unsigned long long u64;

static void mulhilo64(u64 a, u64 b, u64 *hi, u64 *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (u64)(p >> 64);
    *lo = (u64)p;
}

void orc_philox4x64(const u64 ctr[4], const u64 key[2], u64 out[4])
{
    const u64 M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const u64 W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    u64 x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        u64 h0, l0, h1, l1;
        mulhilo64(M0, x0, &h0, &l0);
        mulhilo64(M1, x2, &h1, &l1);
        const u64 y0 = h1 ^ x1 ^ k0, y1 = l1, y2 = h0 ^ x3 ^ k1, y3 = l0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/*
 * Four independent standard normal numbers for (site, purpose) of the current
 * step: key (seed, rep), counter (site, step, purpose, 0); the four 64-bit words
 * give two Box-Muller pairs, the radius from u1 = (top 53 bits + 1) 2^-53 in (0, 1]
 * and the angle 2 pi u2 with u2 = (top 53 bits) 2^-53 in [0, 1).
 * Purposes: 0-3 the LB modes 4-18 (mode k takes number k - 4), 4 + I the bonds
 * (x, y, z) of species I.
 */
void orc_normals(const orc_sys *s, u64 site_index, u64 purpose, double z[4])
{
    const u64 ctr[4] = {site_index, s->step, purpose, 0ULL}, key[2] = {s->seed, s->rep};
    u64 r[4];
    orc_philox4x64(ctr, key, r);
    const double two53 = 1.0 / 9007199254740992.0;
    for (int p = 0; p < 2; ++p) {
        const double u1 = (double)((r[2 * p] >> 11) + 1ULL) * two53;
        const double u2 = (double)(r[2 * p + 1] >> 11) * two53;
        const double rad = sqrt(-2.0 * log(u1)), ang = 6.283185307179586 * u2;
        z[2 * p] = rad * cos(ang);
        z[2 * p + 1] = rad * sin(ang);
    }
}

/* D3Q19 velocity set (rest, 6 faces, 12 edges) and weights of eq. 11. */
static const int CV[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double wgt(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

void orc_lb_velocity(int i, int c[3])
{
    c[0] = CV[i][0];
    c[1] = CV[i][1];
    c[2] = CV[i][2];
}

/* Second-order equilibrium, eq. 11, with c = 1 so c_s^2 = 1/3. */
static double equilibrium(int i, double rho, const double u[3])
{
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double cs2 = 1.0 / 3.0;
    return rho * wgt(i) * (1.0 + cu / cs2 + 0.5 * cu * cu / (cs2 * cs2) - 0.5 * uu / cs2);
}

void orc_lb_equilibrium(double rho, const double u[3], double neq[19])
{
    for (int i = 0; i < 19; ++i) neq[i] = equilibrium(i, rho, u);
}

/* Basis vector e_k of Table 1 evaluated at velocity c_i (c = 1). */
static double basis(int k, int i)
{
    double cx = CV[i][0], cy = CV[i][1], cz = CV[i][2];
    double c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0: return 1.0;
    case 1: return cx;
    case 2: return cy;
    case 3: return cz;
    case 4: return c2 - 1.0;
    case 5: return cx * cx - cy * cy;
    case 6: return c2 - 3.0 * cz * cz;
    case 7: return cx * cy;
    case 8: return cx * cz;
    case 9: return cy * cz;
    case 10: return (3.0 * c2 - 5.0) * cx;
    case 11: return (3.0 * c2 - 5.0) * cy;
    case 12: return (3.0 * c2 - 5.0) * cz;
    case 13: return (cy * cy - cz * cz) * cx;
    case 14: return (cz * cz - cx * cx) * cy;
    case 15: return (cx * cx - cy * cy) * cz;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (cx * cx - cy * cy);
    default: return (2.0 * c2 - 3.0) * (c2 - 3.0 * cz * cz);
    }
}

double orc_mrt_basis(int k, int i) { return basis(k, i); }

/*
 * One collision at a site.  n: 19 pre-collision populations; f: force density;
 * on exit nout holds the post-collision populations and rho, u the moments of
 * eq. 9 (u includes the half-force shift).
 * lb_mode 0: BGK, L_ij = -delta_ij / tau, with the forcing term
 *   F_i = (1 - 1/(2 tau)) w_i [ (c_i - u).f / c_s^2 + (c_i.u)(c_i.f) / c_s^4 ]
 * lb_mode 1: the multiple-relaxation-time scheme of eq. 12-14 with the basis
 *   of Table 1, gamma_0..3 = 1, gamma_4 = gamma_b, gamma_5..9 = gamma_s, the
 *   kinetic (ghost) modes gamma_10..18 = gamma_ghost, and no mode noise.
 */
static void lb_noise(const orc_sys *s, long r, double rho, double nout[19]);

static void collide(const orc_sys *s, long r, const double n[19], const double f[3], double nout[19],
                    double *rho_out, double u[3])
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
        rho += n[i];
        for (int a = 0; a < 3; ++a) j[a] += n[i] * CV[i][a];
    }
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * f[a]) / rho;
    *rho_out = rho;
    double cs2 = 1.0 / 3.0;
    if (s->lb_mode == 0) {
        double tau = s->tau;
        for (int i = 0; i < 19; ++i) {
            double ci[3] = {CV[i][0], CV[i][1], CV[i][2]};
            double cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2];
            double cf = ci[0] * f[0] + ci[1] * f[1] + ci[2] * f[2];
            double cmu_f = (ci[0] - u[0]) * f[0] + (ci[1] - u[1]) * f[1] + (ci[2] - u[2]) * f[2];
            double F = (1.0 - 0.5 / tau) * wgt(i) * (cmu_f / cs2 + cu * cf / (cs2 * cs2));
            double neq = equilibrium(i, rho, u);
            nout[i] = n[i] - (n[i] - neq) / tau + F;
        }
        if (s->noise & 2) lb_noise(s, r, rho, nout);
        return;
    }
    double gk[19];
    for (int k = 0; k < 19; ++k)
        gk[k] = k <= 3 ? 1.0 : (k == 4 ? s->gamma_b : (k <= 9 ? s->gamma_s : s->gamma_ghost));
    double uf = u[0] * f[0] + u[1] * f[1] + u[2] * f[2];
    double Sig[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double dab = (a == b) ? 1.0 : 0.0;
            Sig[a][b] = 0.5 * (1.0 + s->gamma_s) * (u[a] * f[b] + u[b] * f[a] - 2.0 / 3.0 * uf * dab) +
                        1.0 / 3.0 * (1.0 + s->gamma_b) * uf * dab;
        }
    double neq[19], dfi[19];
    for (int i = 0; i < 19; ++i) {
        neq[i] = equilibrium(i, rho, u);
        double fc = 0.0, ss = 0.0;
        for (int a = 0; a < 3; ++a) {
            fc += f[a] * CV[i][a];
            for (int b = 0; b < 3; ++b)
                ss += Sig[a][b] * (CV[i][a] * CV[i][b] - cs2 * (a == b ? 1.0 : 0.0));
        }
        dfi[i] = wgt(i) / cs2 * (fc + ss / (2.0 * cs2));
    }
    double mstar[19], bk[19];
    for (int k = 0; k < 19; ++k) {
        double m = 0.0, mf = 0.0, b = 0.0;
        for (int i = 0; i < 19; ++i) {
            double e = basis(k, i);
            m += (n[i] - neq[i]) * e;
            mf += dfi[i] * e;
            b += wgt(i) * e * e;
        }
        mstar[k] = gk[k] * m + mf;
        bk[k] = b;
    }
    for (int i = 0; i < 19; ++i) {
        double acc = 0.0;
        for (int k = 0; k < 19; ++k) acc += mstar[k] * basis(k, i) / bk[k];
        nout[i] = neq[i] + wgt(i) * acc;
    }
    if (s->noise & 2) lb_noise(s, r, rho, nout);
}

/*
 * Mode noise of eq. 13 added to the post-collision populations of site r: mode
 * k >= 4 of the Table 1 basis receives phi_k r_k with
 * phi_k = sqrt(rho kT b_k (1 - gamma_k^2) / c_s^2) (h = 1), which the reconstruction
 * n_i = n_eq + w_i sum_k m_k e_ki / b_k carries to the populations.  gamma_k as in
 * the collision (BGK: 1 - 1/tau for every non-conserved mode).  kT in LB units is
 * dt^2 / Omega (mass unit m0 h^3 / v0 with LB density 1, time unit the step, and
 * m0 = kT tau^2 / h^2 of sec. 3).  A negative density gives no noise.
 */
static void lb_noise(const orc_sys *s, long r, double rho, double nout[19])
{
    const double kT = s->dt * s->dt / s->omega, cs2 = 1.0 / 3.0;
    double z[16];
    for (int p = 0; p < 4; ++p) orc_normals(s, (u64)r, (u64)p, z + 4 * p);
    double amp[19];
    for (int k = 4; k < 19; ++k) {
        double g = s->lb_mode == 0 ? 1.0 - 1.0 / s->tau
                                   : (k == 4 ? s->gamma_b : (k <= 9 ? s->gamma_s : s->gamma_ghost));
        double b = 0.0;
        for (int i = 0; i < 19; ++i) b += wgt(i) * basis(k, i) * basis(k, i);
        const double phik = sqrt(fmax(rho, 0.0) * kT * b * (1.0 - g * g) / cs2);
        amp[k] = phik * z[k - 4] / b;
    }
    for (int i = 0; i < 19; ++i) {
        double acc = 0.0;
        for (int k = 4; k < 19; ++k) acc += amp[k] * basis(k, i);
        nout[i] += wgt(i) * acc;
    }
}

/*
 * One lattice-Boltzmann step, eq. 10: collide at every site, then stream each
 * population one lattice step along its velocity (periodic).
 * n, nout: [19][V] (pre-collision, before and after the step); f: [3][V] or
 * NULL for no force; rho: [V] and u: [3][V] (may be NULL) receive the moments
 * of eq. 9 of the pre-collision state.
 */
void orc_lb_step(const orc_sys *s, const double *n, const double *f, double *nout, double *rho, double *u)
{
    long V = vol(s);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->Lz; ++z)
        for (int y = 0; y < s->Ly; ++y)
            for (int x = 0; x < s->Lx; ++x) {
                long r = site(s, x, y, z);
                double nl[19], ns_[19], fl[3] = {0.0, 0.0, 0.0}, rl, ul[3];
                for (int i = 0; i < 19; ++i) nl[i] = n[(long)i * V + r];
                if (f)
                    for (int a = 0; a < 3; ++a) fl[a] = f[(long)a * V + r];
                collide(s, r, nl, fl, ns_, &rl, ul);
                for (int i = 0; i < 19; ++i)
                    nout[(long)i * V + site(s, x + CV[i][0], y + CV[i][1], z + CV[i][2])] = ns_[i];
                if (rho) rho[r] = rl;
                if (u)
                    for (int a = 0; a < 3; ++a) u[(long)a * V + r] = ul[a];
            }
}

/*
 * One explicit update of the convection-diffusion equation (eq. 3, noise
 * off, M = kT = 1) in conservative flux form.  The paper integrates diffusion
 * with Crank-Nicolson and convection with two-step Lax-Wendroff; reading: an
 * explicit step for the diffusive flux (stable for the small dt used here)
 * and the Richtmyer two-step Lax-Wendroff flux for convection, per axis.
 * For the face between r and r + e_alpha:
 *   J^D = -1/2 (phi(r) + phi(r+e)) (mu(r+e) - mu(r))
 *   phi_half = 1/2 (phi(r) + phi(r+e)) - 1/2 ((phi u_a)(r+e) - (phi u_a)(r))
 *   J^C = phi_half * 1/2 (u_a(r) + u_a(r+e))
 *   phi_new(r) = phi(r) - sum_a [ dt (J^D(r+) - J^D(r-)) + (J^C(r+) - J^C(r-)) ]
 * u is the LB velocity, i.e. the displacement per step in lattice units.
 * phi, mu, phi_out: [species][V]; u: [3][V] or NULL (no convection).
 *
 * Composition noise (noise bit 0), eq. 5 with M = kT = 1: the cited algorithm for
 * xi_I is not reproduced in the paper; reading: a random flux on every bond, the one
 * between r and r + e_a owned by r,
 *   J^N = sqrt(2 dt max(phi_bond, 0) / Omega) g,  phi_bond = (phi(r) + phi(r+e)) / 2,
 * with g the species' standard normal number for that bond, added to the face flux.
 * Its divergence has the covariance (2 dt / Omega) (-div phi grad) of eq. 5 integrated
 * over a step (delta(r - r') = 1 / h^3 on the lattice and phi = rho v0 give the factor
 * v0 / h^3 = 1 / Omega), and it conserves each species' amount exactly.
 */
void orc_cd_update(const orc_sys *s, const double *phi, const double *mu, const double *u, double *phi_out)
{
    long V = vol(s);
    int ns = nsp(s);
    for (int I = 0; I < ns; ++I) {
        const double *p = phi + (long)I * V;
        const double *m = mu + (long)I * V;
        for (int z = 0; z < s->Lz; ++z)
            for (int y = 0; y < s->Ly; ++y)
                for (int x = 0; x < s->Lx; ++x) {
                    long r = site(s, x, y, z);
                    double div = 0.0;
                    double zr[4] = {0.0, 0.0, 0.0, 0.0};
                    if (s->noise & 1) orc_normals(s, (u64)r, (u64)(4 + I), zr);
                    for (int a = 0; a < 3; ++a) {
                        int e[3] = {a == 0, a == 1, a == 2};
                        /* faces r - e/2 (between rm and r) and r + e/2 (between r and rp) */
                        long rm = site(s, x - e[0], y - e[1], z - e[2]);
                        long rp = site(s, x + e[0], y + e[1], z + e[2]);
                        long lo[2] = {rm, r}, hi[2] = {r, rp};
                        double J[2];
                        for (int side = 0; side < 2; ++side) {
                            long A = lo[side], B = hi[side];
                            double jd = -0.5 * (p[A] + p[B]) * (m[B] - m[A]);
                            double jc = 0.0;
                            if (u) {
                                double ua = u[(long)a * V + A], ub = u[(long)a * V + B];
                                double half = 0.5 * (p[A] + p[B]) - 0.5 * (p[B] * ub - p[A] * ua);
                                jc = half * 0.5 * (ua + ub);
                            }
                            J[side] = s->dt * jd + jc;
                            if (s->noise & 1) {
                                /* the bond's number belongs to its lower site A */
                                double g = zr[a];
                                if (side == 0) {
                                    double zo[4];
                                    orc_normals(s, (u64)A, (u64)(4 + I), zo);
                                    g = zo[a];
                                }
                                J[side] += sqrt(2.0 * s->dt * fmax(0.5 * (p[A] + p[B]), 0.0) / s->omega) * g;
                            }
                        }
                        div += J[1] - J[0];
                    }
                    phi_out[(long)I * V + r] = p[r] - div;
                }
    }
}

/*
 * One coupled step (paper section 2: LB steps alternate with steps of eq. 3
 * at equal time step; each step of eq. 3 first determines the fields).
 * Reading of the order inside a step:
 *   1. invert phi^n -> w^n (w holds the warm start on entry);
 *   2. mu^n and the force f^n from phi^n, w^n;
 *   3. LB: moments of the pre-collision state with the half-force shift give
 *      u^n; collide and stream (skipped, u = 0, when hydro is off);
 *   4. convection-diffusion update phi^n -> phi^{n+1} with mu^n and u^n.
 * phi, w: [species][V] (updated in place); n: [19][V] (updated in place, may
 * be NULL when hydro is off).  u_out [3][V], rho_out [V] optional.
 * Returns the inversion status.
 */
int orc_step(const orc_sys *s, double *phi, double *w, double *n, double tol, int max_iter,
             int fixed_iters, orc_invert_stats *st, double *u_out, double *rho_out)
{
    long V = vol(s);
    int ns = nsp(s);
    int rc = orc_invert(s, phi, w, tol, max_iter, fixed_iters, st);
    if (rc < 0) return rc;
    double *mu = malloc(sizeof(double) * V * ns);
    double *f = malloc(sizeof(double) * V * 3);
    double *u = calloc((size_t)V * 3, sizeof(double));
    double *rho = malloc(sizeof(double) * V);
    double *nn = (s->hydro && n) ? malloc(sizeof(double) * V * 19) : NULL;
    double *pn = malloc(sizeof(double) * V * ns);
    orc_mu_force(s, phi, w, mu, f);
    if (s->hydro && n) {
        orc_lb_step(s, n, f, nn, rho, u);
        memcpy(n, nn, sizeof(double) * V * 19);
    } else {
        for (long r = 0; r < V; ++r) rho[r] = 1.0;
    }
    orc_cd_update(s, phi, mu, (s->hydro && n) ? u : NULL, pn);
    memcpy(phi, pn, sizeof(double) * V * ns);
    if (u_out) memcpy(u_out, u, sizeof(double) * V * 3);
    if (rho_out) memcpy(rho_out, rho, sizeof(double) * V);
    free(mu); free(f); free(u); free(rho); free(nn); free(pn);
    return rc;
}

/* Threads the site loops use (1 in the plain build). */
#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
#else
int orc_threads(void) { return 1; }
#endif
