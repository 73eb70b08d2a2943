/*
 * Host-side checks of the C ABI for the sanitizer build (AddressSanitizer and
 * UndefinedBehaviorSanitizer on the library's host code): every entry point
 * is called with the arguments its validation refuses before any GPU work,
 * and the returned status and message are checked.  Needs no GPU.  Exit
 * status 0 when every check holds.
 */
#include <stdio.h>
#include <string.h>

#include "mk.h"

static int failures = 0;

static void expect(int cond, const char* what) {
    if (!cond) {
        fprintf(stderr, "host_check: FAILED %s\n", what);
        ++failures;
    }
}

static mk_plan_desc good(void) {
    mk_plan_desc d;
    memset(&d, 0, sizeof(d));
    d.nr = 8;
    d.ns = 8;
    d.nt = 64;
    d.iw_lo = 0;
    d.iw_hi = 32;
    d.nf_max = 1;
    d.dt = 0.004;
    d.dx = 10.0;
    d.rprec = MK_R_C64;
    return d;
}

static void plan_refused(mk_plan_desc d, mk_status want, const char* what) {
    mk_plan_t p = (mk_plan_t)0x1;
    const mk_status st = mk_plan(&d, &p);
    expect(st == want, what);
    expect(p == NULL, "plan handle cleared on failure");
    expect(strncmp(mk_last_error(NULL), "mk_plan", 7) == 0, "mk_plan message");
}

int main(void) {
    for (int s = 0; s < 7; ++s) expect(mk_strerror(s)[0] != '\0', "strerror");
    expect(strcmp(mk_strerror(99), "unknown status") == 0, "strerror of an unknown status");
    expect(strcmp(mk_strerror(-1), "unknown status") == 0, "strerror of a negative status");

    mk_plan_t p = NULL;
    expect(mk_plan(NULL, &p) == MK_ERR_ARG, "mk_plan(NULL desc)");
    mk_plan_desc d = good();
    expect(mk_plan(&d, NULL) == MK_ERR_ARG, "mk_plan(NULL out)");

    d = good(); d.ns = 9; plan_refused(d, MK_ERR_ARG, "nr != ns");
    d = good(); d.nt = 48; plan_refused(d, MK_ERR_ARG, "nt not a power of two");
    d = good(); d.nt = 8192; d.iw_hi = 100; plan_refused(d, MK_ERR_ARG, "nt above 4096");
    d = good(); d.iw_lo = 5; d.iw_hi = 4; plan_refused(d, MK_ERR_ARG, "empty band");
    d = good(); d.iw_hi = 33; plan_refused(d, MK_ERR_ARG, "band above nt/2");
    d = good(); d.nf_max = 0; plan_refused(d, MK_ERR_ARG, "nf_max 0");
    d = good(); d.dt = 0.0; plan_refused(d, MK_ERR_ARG, "dt 0");
    d = good(); d.rprec = 7; plan_refused(d, MK_ERR_ARG, "unknown rprec");
    d = good(); d.flags = 0x100; plan_refused(d, MK_ERR_ARG, "unknown flag");
    d = good(); d.ns = d.nr = 5000; plan_refused(d, MK_ERR_UNSUPPORTED, "ns above 4096");
    d = good(); d.r_dev_bytes = 4095; plan_refused(d, MK_ERR_ARG, "cap below two bins of R");
    d = good(); d.r_dev_bytes = 8192; d.flags = MK_FLAG_GRAPH; plan_refused(d, MK_ERR_UNSUPPORTED, "graph + streamed R");

    /* every plan call refuses a NULL plan */
    float f = 0.f;
    double g = 0.0;
    int32_t i = 0;
    int64_t l = 0;
    size_t z = 0;
    char blob[64];
    expect(mk_load_R(NULL, &f, 0) == MK_ERR_ARG, "mk_load_R(NULL)");
    expect(mk_set_focal(NULL, 1, &f, &i, 0, NULL, 0) == MK_ERR_ARG, "mk_set_focal(NULL)");
    expect(mk_iterate(NULL, 1, NULL) == MK_ERR_ARG, "mk_iterate(NULL)");
    expect(mk_iterate_tol(NULL, 1e-3, 4, &i, &g) == MK_ERR_ARG, "mk_iterate_tol(NULL)");
    expect(mk_get(NULL, MK_F1PLUS, &f, 0) == MK_ERR_ARG, "mk_get(NULL)");
    expect(mk_image(NULL, &g) == MK_ERR_ARG, "mk_image(NULL)");
    expect(mk_tune(NULL, -1) == MK_ERR_ARG, "mk_tune(NULL)");
    expect(mk_contract_variant(NULL, 1, &i) == MK_ERR_ARG, "mk_contract_variant(NULL)");
    expect(mk_passes(NULL, &i) == MK_ERR_ARG, "mk_passes(NULL)");
    expect(mk_profile(NULL, 0, &g, &l, 0) == MK_ERR_ARG, "mk_profile(NULL)");
    expect(mk_tail_record(NULL, 4, 64) == MK_ERR_ARG, "mk_tail_record(NULL)");
    expect(mk_tail_load(NULL, &f, 1) == MK_ERR_ARG, "mk_tail_load(NULL)");
    expect(mk_tail_history(NULL, &f, 0) == MK_ERR_ARG, "mk_tail_history(NULL)");
    expect(mk_tail_apply(NULL, 0, &g) == MK_ERR_ARG, "mk_tail_apply(NULL)");
    expect(mk_state_bytes(NULL, &z) == MK_ERR_ARG, "mk_state_bytes(NULL)");
    expect(mk_get_state(NULL, blob, sizeof(blob)) == MK_ERR_ARG, "mk_get_state(NULL)");
    expect(mk_set_state(NULL, blob, sizeof(blob)) == MK_ERR_ARG, "mk_set_state(NULL)");
    expect(mk_destroy(NULL) == MK_OK, "mk_destroy(NULL) is a no-op");

    /* network calls: sizes and NULL pointers are refused before any launch */
    expect(mk_net_param_count(4, 16) > 0, "param count");
    expect(mk_net_param_count(0, 16) == -1 && mk_net_param_count(4, 0) == -1 && mk_net_param_count(17, 16) == -1,
           "param count out of range");
    expect(mk_net_forward(NULL, &f, 1, 4, 16, 8, &f, &f, NULL) == MK_ERR_ARG, "mk_net_forward(NULL)");
    expect(mk_net_forward(&f, &f, 0, 4, 16, 8, &f, &f, NULL) == MK_ERR_ARG, "mk_net_forward(N = 0)");
    expect(mk_net_backward(&f, &f, &f, &f, 1, 4, 200, 8, &f, &f, NULL) == MK_ERR_ARG, "mk_net_backward(hidden)");
    expect(mk_net_loss(&f, &f, &f, 1, 8, 1.f, &f, &g, &g, 0, NULL) == MK_ERR_ARG, "mk_net_loss(nparts 0)");
    expect(mk_net_loss_noalloc(&f, &f, &f, 1, 8, 1.f, &f, &g, 1025, NULL) == MK_ERR_ARG,
           "mk_net_loss_noalloc(nparts above the array)");
    expect(mk_net_loss_noalloc(&f, &f, &f, 1, 8, 0.f, &f, &g, 4, NULL) == MK_ERR_ARG, "mk_net_loss_noalloc(count)");
    expect(mk_net_adam(&f, &f, &f, &f, &f, 1, 0, 1e-3f, 0.9f, 0.999f, 1e-8f, NULL) == MK_ERR_ARG,
           "mk_net_adam(step 0)");
    expect(mk_net_round(NULL, &f, 1, NULL) == MK_ERR_ARG, "mk_net_round(NULL)");
    expect(mk_net_last_error()[0] != '\0', "network message");

    if (failures == 0) printf("host_check: all checks passed\n");
    return failures == 0 ? 0 : 1;
}
