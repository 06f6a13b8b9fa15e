/* Host sanitizer run of the C ABI: the library's host code built with
 * -fsanitize=address,undefined (device code not built) and driven through every entry
 * point that needs no device work: argument checks with null handles and pointers, the
 * paired-sweep schedule for every chain length and launch, hsf_create and hsf_net_create
 * with bad parameters, and with good ones the failure path when no GPU is present
 * (partially created contexts are torn down).  Exit status 0 and a last line
 * "abi driver ok" when every check held. */
#include <stdio.h>
#include <string.h>

#include "hsf.h"

static int failures = 0;

#define CHECK(cond)                                                           \
    do {                                                                      \
        if (!(cond)) {                                                        \
            printf("check failed, line %d: %s\n", __LINE__, #cond);           \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static hsf_params melt(int L)
{
    hsf_params p;
    memset(&p, 0, sizeof p);
    p.Lx = L; p.Ly = L + 1; p.Lz = L + 2;
    p.n_beads = 4;
    p.types[2] = 1; p.types[3] = 1;
    p.a = 1.1543;
    p.chi[0][1] = p.chi[1][0] = 0.5;
    p.kappa = 10.0; p.dt = 0.01; p.tau = 1.0; p.hydro = 1;
    return p;
}

int main(void)
{
    /* the paired schedule: every launch of every chain length, then bad arguments */
    int out[8];
    long long total = 0;
    for (int n = 2; n <= HSF_MAX_BEADS; ++n)
        for (int j = 1; j <= n; ++j) {
            CHECK(hsf_paired_schedule(n, j, out) == HSF_OK);
            total += out[0] + out[1];
        }
    CHECK(hsf_paired_schedule(1, 1, out) == HSF_EINVAL);
    CHECK(hsf_paired_schedule(8, 0, out) == HSF_EINVAL);
    CHECK(hsf_paired_schedule(8, 9, out) == HSF_EINVAL);
    CHECK(hsf_paired_schedule(HSF_MAX_BEADS + 1, 1, out) == HSF_EINVAL);
    CHECK(hsf_paired_schedule(8, 1, NULL) == HSF_EINVAL);

    /* null handles and pointers */
    double d = 0.0;
    long long ll = 0;
    int iv = 0;
    hsf_invert_stats st;
    hsf_step_record rec;
    hsf_cn_stats cs;
    unsigned long long ul = 0;
    int cfg[4] = {32, 8, 2, 0};
    CHECK(hsf_create(NULL, 1, NULL) == HSF_EINVAL);
    hsf_destroy(NULL);
    (void)hsf_last_error(NULL);
    CHECK(hsf_set_stream(NULL, NULL) != HSF_OK);
    (void)hsf_total_sites(NULL);
    (void)hsf_site_offset(NULL, 0);
    (void)hsf_field_offset(NULL, 0);
    (void)hsf_num_species(NULL);
    CHECK(hsf_set_fields(NULL, &d, HSF_HOST) != HSF_OK);
    CHECK(hsf_get_fields(NULL, &d, HSF_HOST) != HSF_OK);
    CHECK(hsf_set_densities(NULL, &d, HSF_HOST) != HSF_OK);
    CHECK(hsf_get_densities(NULL, &d, HSF_HOST) != HSF_OK);
    CHECK(hsf_evaluate(NULL, &d, &d, HSF_HOST) != HSF_OK);
    CHECK(hsf_observables(NULL, &d, &d, &d) != HSF_OK);
    CHECK(hsf_invert(NULL, 1e-8, 10, HSF_WARM_CURRENT, &st) != HSF_OK);
    CHECK(hsf_mu_force(NULL, &d, &d, HSF_HOST) != HSF_OK);
    CHECK(hsf_set_lb(NULL, &d, HSF_HOST) != HSF_OK);
    CHECK(hsf_get_lb(NULL, &d, HSF_HOST) != HSF_OK);
    CHECK(hsf_lb_advance(NULL, 1, NULL, HSF_HOST) != HSF_OK);
    CHECK(hsf_get_flow(NULL, &d, &d, HSF_HOST) != HSF_OK);
    CHECK(hsf_cd_advance(NULL, &d, NULL, HSF_HOST) != HSF_OK);
    CHECK(hsf_step(NULL, 1, 1e-8, 10, &st, &ll) != HSF_OK);
    (void)hsf_state_size(NULL);
    CHECK(hsf_get_state(NULL, &d, 8) != HSF_OK);
    CHECK(hsf_set_state(NULL, &d, 8) != HSF_OK);
    CHECK(hsf_set_integrator(NULL, 1, 1e-8, 10, 20) != HSF_OK);
    CHECK(hsf_get_cn_stats(NULL, &cs) != HSF_OK);
    CHECK(hsf_set_noise(NULL, 3, 400.0, 1, 0) != HSF_OK);
    CHECK(hsf_get_noise_step(NULL, &ul) != HSF_OK);
    CHECK(hsf_set_hydro(NULL, 1) != HSF_OK);
    CHECK(hsf_set_solver(NULL, 1) != HSF_OK);
    CHECK(hsf_get_work(NULL, &ll, &d, 0) != HSF_OK);
    CHECK(hsf_set_tile(NULL, cfg) != HSF_OK);
    CHECK(hsf_get_tile(NULL, cfg) != HSF_OK);
    CHECK(hsf_autotune(NULL, 1, &d) != HSF_OK);
    CHECK(hsf_set_warm(NULL, HSF_WARM_EXTRAP) != HSF_OK);
    CHECK(hsf_attach_net(NULL, NULL) != HSF_OK);
    CHECK(hsf_set_net_gate(NULL, 2) != HSF_OK);
    CHECK(hsf_set_timing(NULL, 1) != HSF_OK);
    CHECK(hsf_get_timing(NULL, &d, &ll) != HSF_OK);
    CHECK(hsf_set_step_log(NULL, 1) != HSF_OK);
    CHECK(hsf_read_step_log(NULL, &rec, 1, &iv) != HSF_OK);
    hsf_net_destroy(NULL);
    (void)hsf_net_last_error(NULL);
    (void)hsf_net_num_params(NULL);
    CHECK(hsf_net_set_stream(NULL, NULL) != HSF_OK);
    CHECK(hsf_net_set_params(NULL, NULL, HSF_HOST) != HSF_OK);
    CHECK(hsf_net_get_params(NULL, NULL, HSF_HOST) != HSF_OK);
    CHECK(hsf_net_set_input_norm(NULL, NULL, NULL) != HSF_OK);
    CHECK(hsf_net_set_output_scale(NULL, NULL) != HSF_OK);
    CHECK(hsf_net_forward(NULL, NULL, NULL, 1, 8, HSF_HOST) != HSF_OK);
    CHECK(hsf_net_loss_grad(NULL, NULL, NULL, 1, 8, &d, NULL, HSF_HOST) != HSF_OK);
    CHECK(hsf_net_train_step(NULL, NULL, NULL, 1, 8, 1e-3f, &d, HSF_HOST) != HSF_OK);
    CHECK(hsf_net_make_sample(NULL, NULL, NULL, NULL, NULL, NULL, NULL, 2, 8, 1, NULL, NULL) != HSF_OK);
    CHECK(hsf_net_affine(NULL, NULL, 1, 1, 8, NULL, NULL) != HSF_OK);
    CHECK(hsf_net_channel_moments(NULL, NULL, 1, 1, 8, &d, &d) != HSF_OK);

    /* bad parameters: refused before any device work */
    hsf_ctx *ctx = NULL;
    hsf_params bad[2];
    bad[0] = melt(6);
    bad[0].Lx = 0;
    CHECK(hsf_create(bad, 1, &ctx) == HSF_EINVAL && ctx == NULL);
    bad[0] = melt(6);
    bad[0].n_beads = 0;
    CHECK(hsf_create(bad, 1, &ctx) == HSF_EINVAL && ctx == NULL);
    bad[0] = melt(6);
    bad[0].n_beads = HSF_MAX_BEADS + 1;
    CHECK(hsf_create(bad, 1, &ctx) == HSF_EINVAL && ctx == NULL);
    bad[0] = melt(6);
    bad[0].types[1] = 7;
    CHECK(hsf_create(bad, 1, &ctx) == HSF_EINVAL && ctx == NULL);
    bad[0] = melt(6);
    bad[0].tau = 0.4;
    CHECK(hsf_create(bad, 1, &ctx) == HSF_EINVAL && ctx == NULL);
    bad[0] = melt(6);
    bad[0].Lx = 65536; bad[0].Ly = 65536; bad[0].Lz = 2;
    CHECK(hsf_create(bad, 1, &ctx) == HSF_EINVAL && ctx == NULL);
    bad[0] = melt(6);
    bad[1] = melt(7);
    bad[1].has_solvent = 1;   /* replicas must share the chain and species */
    CHECK(hsf_create(bad, 2, &ctx) == HSF_EINVAL && ctx == NULL);
    CHECK(hsf_create(bad, 0, &ctx) == HSF_EINVAL && ctx == NULL);
    hsf_net *net = NULL;
    int widths[4] = {8, 16, 0, 0};
    CHECK(hsf_net_create(0, 2, widths, 1, &net) == HSF_EINVAL && net == NULL);
    int wbad[4] = {0, 0, 0, 0};
    CHECK(hsf_net_create(4, 2, wbad, 1, &net) == HSF_EINVAL && net == NULL);

    /* good parameters: without a GPU creation fails cleanly; with one the context works
     * and is destroyed */
    hsf_params good[2] = {melt(6), melt(5)};
    int rc = hsf_create(good, 2, &ctx);
    printf("hsf_create: %d\n", rc);
    if (rc == HSF_OK) {
        CHECK(ctx != NULL);
        CHECK(hsf_total_sites(ctx) == 6LL * 7 * 8 + 5LL * 6 * 7);
        hsf_destroy(ctx);
    } else {
        CHECK(ctx == NULL);
        double q = 0.0;
        double buf[8];
        CHECK(hsf_evaluate_static(&good[0], buf, buf, buf, &q, NULL) != HSF_OK);
    }
    rc = hsf_net_create(4, 2, widths, 1, &net);
    printf("hsf_net_create: %d\n", rc);
    if (rc == HSF_OK) hsf_net_destroy(net);
    else CHECK(net == NULL);
    double q = 0.0, buf[8];
    hsf_params sbad = melt(6);
    sbad.n_beads = 0;
    CHECK(hsf_evaluate_static(&sbad, buf, buf, buf, &q, NULL) == HSF_EINVAL);
    CHECK(hsf_evaluate_static(NULL, buf, buf, buf, &q, NULL) == HSF_EINVAL);

    printf("schedule checksum %lld, failures %d\n", total, failures);
    if (failures) return 1;
    printf("abi driver ok\n");
    return 0;
}
