/* Host sanitizer run of the oracle: every function of oracle/hsf_oracle.c on small
 * ragged boxes (a solution with both noises, BGK and MRT, plain and preconditioned
 * inversion; a melt without flow), built with -fsanitize=address,undefined.  The
 * oracle's source is included whole, so its internal helpers are instrumented too.
 * Exit status 0 and a last line "oracle driver ok" when every call returned. */
#include "../../oracle/hsf_oracle.c"

#include <stdio.h>

/* Target densities the chain can reach: the mean of each block species is its share of
 * the chain times the copolymer fraction, with a small mean-free modulation. */
static void fill_targets(const orc_sys *s, double *phi)
{
    long V = vol(s);
    int nA = 0;
    for (int k = 0; k < s->N; ++k) nA += s->types[k] == 0;
    double phip = s->has_solvent ? 0.3 : 1.0, fA = phip * nA / s->N;
    for (long i = 0; i < V; ++i) {
        double e = 0.01 * (double)((i * 7919) % 13 - 6) / 6.0;
        if (i == V - 1) e = 0.0;
        phi[i] = fA + e;
        phi[V + i] = phip - fA - e;
        if (s->has_solvent) phi[2 * V + i] = 1.0 - phip;
    }
    double m = 0.0;   /* make the modulation mean-free */
    for (long i = 0; i < V; ++i) m += phi[i] - fA;
    m /= (double)V;
    for (long i = 0; i < V; ++i) {
        phi[i] -= m;
        phi[V + i] += m;
    }
}

static int run_system(orc_sys *s, int solvent)
{
    long V = vol(s);
    int ns = nsp(s);
    double *phi = calloc((size_t)ns * V, sizeof(double)), *w = calloc((size_t)ns * V, sizeof(double));
    double *out = calloc((size_t)ns * V, sizeof(double)), *mu = calloc((size_t)ns * V, sizeof(double));
    double *f = calloc((size_t)3 * V, sizeof(double)), *u = calloc((size_t)3 * V, sizeof(double));
    double *rho = calloc((size_t)V, sizeof(double)), *n = calloc((size_t)19 * V, sizeof(double));
    double *n2 = calloc((size_t)19 * V, sizeof(double)), *Qs = calloc((size_t)s->N, sizeof(double));
    if (!phi || !w || !out || !mu || !f || !u || !rho || !n || !n2 || !Qs) return 1;
    fill_targets(s, phi);
    double phibar_p = 0.0, phibar_s = 0.0;
    for (long i = 0; i < V; ++i) {
        phibar_p += phi[i] + phi[V + i];
        if (solvent) phibar_s += phi[2 * V + i];
    }
    phibar_p /= (double)V;
    phibar_s /= (double)V;
    orc_invert_stats st;
    for (int pc = 0; pc < 2; ++pc) {
        s->precond = pc;
        memset(w, 0, sizeof(double) * ns * V);
        int rc = orc_invert(s, phi, w, 1e-9, 400, 0, &st);
        printf("invert precond %d: rc %d, %d iterations, residual %.3e\n", pc, rc, st.iterations, st.residual);
        if (rc != 0) return 1;
    }
    double Q = 0.0;
    if (orc_evaluate(s, w, phibar_p, phibar_s, out, &Q, Qs) != 0) return 1;
    printf("Q %.12f, ln Q %.12f\n", Q, orc_log_q(s, w));
    orc_sigma(s, phi, out);
    orc_mu_force(s, phi, w, mu, f);
    double sm = 0.0, ss = 0.0;
    orc_order_params(s, phi, &sm, &ss);
    printf("F %.12f, S_melt %.6f, S_sol %.6f\n", orc_free_energy(s, w, phi), sm, ss);
    for (long i = 0; i < V; ++i) {
        double neq[19], uu[3] = {0.001 * (double)(i % 3), 0.0, -0.001};
        orc_lb_equilibrium(1.0, uu, neq);
        for (int q = 0; q < 19; ++q) n[(long)q * V + i] = neq[q];
    }
    for (int mode = 0; mode < 2; ++mode) {
        s->lb_mode = mode;
        orc_lb_step(s, n, f, n2, rho, u);
        memcpy(n, n2, sizeof(double) * 19 * V);
    }
    s->lb_mode = 0;
    orc_cd_update(s, phi, mu, u, out);
    for (int k = 0; k < 3; ++k) {
        int rc = orc_step(s, phi, w, s->hydro ? n : NULL, 1e-8, 400, 0, &st, u, rho);
        ++s->step;
        printf("step %d: rc %d, %d iterations\n", k, rc, st.iterations);
        if (rc != 0) return 1;
    }
    free(phi); free(w); free(out); free(mu); free(f); free(u); free(rho); free(n); free(n2); free(Qs);
    return 0;
}

int main(void)
{
    orc_sys s;
    memset(&s, 0, sizeof s);
    s.Lx = 5; s.Ly = 4; s.Lz = 3;
    s.N = 4;
    s.types[0] = 0; s.types[1] = 0; s.types[2] = 1; s.types[3] = 1;
    s.n_poly = 2;
    s.has_solvent = 1;
    orc_stencil_weights(1.1543, s.c);
    double chi[3][3] = {{0.0, 0.6, 0.2}, {0.6, 0.0, 0.9}, {0.2, 0.9, 0.0}};
    memcpy(s.chi, chi, sizeof chi);
    s.kappa = 10.0; s.dt = 0.01; s.tau = 0.8;
    s.gamma_s = 0.2; s.gamma_b = -0.1; s.gamma_ghost = 0.05;
    s.hydro = 1; s.noise = 3; s.omega = 400.0; s.seed = 7; s.rep = 1;
    if (run_system(&s, 1)) return 1;

    orc_sys m = s;   /* melt, no flow, no noise, odd chain */
    m.Lx = 3; m.Ly = 5; m.Lz = 2;
    m.N = 5;
    m.types[4] = 1;
    m.has_solvent = 0;
    m.hydro = 0; m.noise = 0;
    if (run_system(&m, 0)) return 1;

    unsigned long long ctr[4] = {~0ULL, ~0ULL, 1, 2}, key[2] = {3, 4}, r[4];
    orc_philox4x64(ctr, key, r);
    double z[4];
    orc_normals(&s, 17, 2, z);
    int c[3];
    double acc = 0.0;
    for (int i = 0; i < 19; ++i) {
        orc_lb_velocity(i, c);
        for (int k = 0; k < 19; ++k) acc += orc_mrt_basis(k, i) * (double)(c[0] + c[1] + c[2]);
    }
    printf("philox %llu, normals %.6f, basis sum %.3f, threads %d\n", r[0], z[0], acc, orc_threads());
    printf("oracle driver ok\n");
    return 0;
}
