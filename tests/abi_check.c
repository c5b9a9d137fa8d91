/* Host-side checks of the C ABI, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer against a host-only build of the library (no
 * device code, no GPU needed): every argument check that rejects a call
 * before it reaches the device, the host-only entry points (mask selection
 * by the sensitivity threshold of Sec. 3.1, the trajectory-length rule of
 * App. C), and an engine set-up that passes every check and then fails at
 * the first device call.  Prints "abi_check ok" and exits 0 when every
 * check passes; the sanitizers abort the run on the first memory or
 * undefined-behaviour error. */

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hmc.h"

static int failures = 0;

#define CHECK(cond, what)                                                        \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, what);     \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

/* A valid 2-3-1 MLP with 13 parameters, one chain selecting 3 of them, and
 * 5 rows of data; each case changes one field. */
typedef struct {
    int32_t widths[3];
    double theta0[13];
    int64_t offs[2];
    int64_t idx[3];
    double x[10], y[5];
    hmc_net_desc net;
    hmc_mask_desc mask;
    hmc_data_desc data;
} setup;

static void base(setup* s) {
    memset(s, 0, sizeof *s);
    s->widths[0] = 2; s->widths[1] = 3; s->widths[2] = 1;
    s->offs[0] = 0; s->offs[1] = 3;
    s->idx[0] = 0; s->idx[1] = 4; s->idx[2] = 7;
    s->net.kind = HMC_MLP;
    s->net.n_widths_a = 3;
    s->net.widths_a = s->widths;
    s->net.theta0 = s->theta0;
    s->net.n_params = 13;
    s->net.prior_sd = 1.0;
    s->net.lik_sd = 1.0;
    s->net.precision = HMC_FP32;
    s->mask.n_chains = 1;
    s->mask.offs = s->offs;
    s->mask.idx = s->idx;
    s->data.x = s->x;
    s->data.y = s->y;
    s->data.n_rows = 5;
}

static void expect_rejected(setup* s, const char* needle) {
    hmc_ctx* ctx = NULL;
    hmc_status st = hmc_init(&ctx, &s->net, &s->mask, &s->data, 0, NULL);
    const char* msg = hmc_last_error(NULL);
    CHECK(st == HMC_EINVAL, needle);
    CHECK(ctx == NULL, needle);
    CHECK(msg && strstr(msg, needle), needle);
}

int main(void) {
    setup s;

    base(&s); s.net.n_params = 12;               expect_rejected(&s, "n_params");
    base(&s); s.idx[1] = 7; s.idx[2] = 4;        expect_rejected(&s, "strictly increasing");
    base(&s); s.idx[2] = 13;                     expect_rejected(&s, "out of range");
    base(&s); s.idx[0] = -1;                     expect_rejected(&s, "out of range");
    base(&s); s.offs[0] = 1;                     expect_rejected(&s, "offs[0]");
    base(&s); s.offs[1] = 0;                     expect_rejected(&s, "selects no entry");
    base(&s); s.net.n_widths_a = 1;              expect_rejected(&s, "widths");
    base(&s); s.widths[1] = 0;                   expect_rejected(&s, "widths");
    base(&s); s.widths[1] = 5000;                expect_rejected(&s, "widths");
    base(&s); s.net.prior_sd = 0.0;              expect_rejected(&s, "prior_sd");
    base(&s); s.net.lik_sd = NAN;                expect_rejected(&s, "lik_sd");
    base(&s); s.net.precision = 7;               expect_rejected(&s, "precision");
    base(&s); s.net.kind = 4;                    expect_rejected(&s, "kind");
    base(&s); s.data.n_rows = 0;                 expect_rejected(&s, "n_rows");
    base(&s); s.data.y = NULL;                   expect_rejected(&s, "x and y");

    /* null descriptors and null engines */
    {
        hmc_ctx* ctx = NULL;
        CHECK(hmc_init(&ctx, NULL, NULL, NULL, 0, NULL) == HMC_EINVAL, "null descriptors");
        CHECK(hmc_init(NULL, NULL, NULL, NULL, 0, NULL) == HMC_EINVAL, "null out");
        double U = 0.0, e = 0.0;
        hmc_info_t info;
        CHECK(hmc_sync(NULL) == HMC_EINVAL, "sync on null");
        CHECK(hmc_grad(NULL, &U, NULL) == HMC_EINVAL, "grad on null");
        CHECK(hmc_adapt(NULL, 1, &e, 1, 0.8, &e) == HMC_EINVAL, "adapt on null");
        CHECK(hmc_set_split(NULL, 64) == HMC_EINVAL, "split on null");
        CHECK(hmc_get_info(NULL, &info) == HMC_EINVAL, "info on null");
        hmc_destroy(NULL);
    }

    /* launch shapes outside the documented sets */
    {
        base(&s);
        hmc_ctx* ctx = NULL;
        hmc_tuning t;
        memset(&t, 0, sizeof t);
        t.rows_a = 24;
        CHECK(hmc_init_tuned(&ctx, &s.net, &s.mask, &s.data, 0, NULL, &t) == HMC_EINVAL, "rows_a 24");
        CHECK(ctx == NULL, "rows_a 24 leaves no engine");
        t.rows_a = 0;
        t.threads = 100;
        CHECK(hmc_init_tuned(&ctx, &s.net, &s.mask, &s.data, 0, NULL, &t) == HMC_EINVAL, "threads 100");
        hmc_tuning best;
        double ms = 0.0;
        CHECK(hmc_autotune(&s.net, &s.mask, &s.data, 0, &best, &ms) == HMC_EINVAL, "autotune reps 0");
        s.net.lik_sd = -1.0;
        CHECK(hmc_autotune(&s.net, &s.mask, &s.data, 3, &best, &ms) == HMC_EINVAL, "autotune lik_sd");
    }

    /* sensitivity pass: a bad network kind is rejected before any device work */
    {
        base(&s);
        s.net.kind = 4;
        double sigma[13], s2[13];
        for (int i = 0; i < 13; ++i) sigma[i] = 0.1;
        CHECK(hmc_sensitivity(&s.net, &s.data, sigma, s2, NULL) == HMC_EINVAL, "sensitivity kind");
        CHECK(strstr(hmc_last_error(NULL), "kind") != NULL, "sensitivity message");
    }

    /* mask selection: the largest count of the most sensitive entries whose
     * share of the summed scores stays within tau, in index order */
    {
        const double s2[6] = {0.5, 4.0, 0.25, 2.0, 1.0, 0.25};   /* total 8 */
        int64_t idx[6], n_sel = -1;
        CHECK(hmc_select_mask(s2, 6, 0.75, idx, &n_sel) == HMC_OK, "select ok");
        /* 4 and 2 make 6/8 = 0.75; adding 1 would pass tau */
        CHECK(n_sel == 2 && idx[0] == 1 && idx[1] == 3, "select set");
        CHECK(hmc_select_mask(s2, 6, 1.5, idx, &n_sel) == HMC_EINVAL, "tau above 1");
        CHECK(hmc_select_mask(s2, 0, 0.5, idx, &n_sel) == HMC_EINVAL, "empty scores");
        const double bad[2] = {1.0, -1.0};
        CHECK(hmc_select_mask(bad, 2, 0.5, idx, &n_sel) == HMC_EINVAL, "negative score");
    }

    /* trajectory length by the rule of App. C: L = pi v / (2 eps), rounded,
     * for the largest of the variances v */
    {
        const double var[3] = {0.25, 1.0, 0.04};
        int32_t L = 0;
        CHECK(hmc_trajectory_length(var, 3, 0, 0.01, &L) == HMC_OK, "length ok");
        CHECK(L == 157, "length of the widest direction");
        CHECK(hmc_trajectory_length(var, 3, 2, 0.01, &L) == HMC_EINVAL, "length mode");
        CHECK(hmc_trajectory_length(var, 3, 0, 0.0, &L) == HMC_EINVAL, "length eps");
        const double neg[1] = {-1.0};
        CHECK(hmc_trajectory_length(neg, 1, 0, 0.01, &L) == HMC_EINVAL, "length variance");
    }

    /* a valid engine description: every check passes, then the first device
     * call fails on a host without a GPU (or the engine is made on a GPU
     * host); either way nothing leaks or overruns */
    {
        base(&s);
        hmc_ctx* ctx = NULL;
        hmc_status st = hmc_init(&ctx, &s.net, &s.mask, &s.data, 1, NULL);
        CHECK(st == HMC_OK || st == HMC_EDEVICE, "valid description");
        CHECK((st == HMC_OK) == (ctx != NULL), "engine only on success");
        if (ctx) hmc_destroy(ctx);
    }

    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("abi_check ok\n");
    return 0;
}
