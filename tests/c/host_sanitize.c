/* Drives the C-ABI host code of libfnt (include/fnt.h), built with
 * AddressSanitizer and UndefinedBehaviorSanitizer for the host side only
 * (tests/test_sanitizers.py), through every argument check and, on a machine
 * with no GPU, through the paths where the HIP runtime reports no device:
 * every call must return an error code (never crash), leave an error text, and
 * free what it took.  Prints "ok" after a clean run. */
#include <stdio.h>
#include <string.h>

#include "../../include/fnt.h"

static int fails = 0;
#define EXPECT(cond)                                                              \
    do {                                                                          \
        if (!(cond)) {                                                            \
            fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, fnt_last_error()); \
            ++fails;                                                              \
        }                                                                         \
    } while (0)

int main(void) {
    fnt_cdc_params cp;
    memset(&cp, 0, sizeof cp);
    cp.ntaps = 8;
    cp.requant_shift = 4;
    fnt_aeq_params ap = {7, 16, 3, 52, 1};
    int8_t x[64 * 4] = {0};
    int16_t taps[256] = {0};
    int16_t out[64 * 4];
    int8_t h[65 * 2] = {0};

    EXPECT(fnt_version() > 0);
    /* argument checks, before any device work */
    EXPECT(fnt_cdc(x, 64, NULL, NULL, NULL, NULL) == FNT_E_INVAL);
    cp.ntaps = 0;
    EXPECT(fnt_cdc(x, 64, &cp, NULL, NULL, NULL) == FNT_E_INVAL);
    cp.ntaps = 33;
    EXPECT(fnt_cdc(x, 64, &cp, NULL, NULL, NULL) == FNT_E_INVAL);
    cp.ntaps = 8;
    cp.taps[3][1] = 40;
    EXPECT(fnt_cdc(x, 64, &cp, NULL, NULL, NULL) == FNT_E_RANGE);
    cp.taps[3][1] = 0;
    cp.decim_phase = 2;
    EXPECT(fnt_cdc(x, 64, &cp, NULL, NULL, NULL) == FNT_E_INVAL);
    cp.decim_phase = 0;
    EXPECT(fnt_cdc(NULL, 64, &cp, NULL, NULL, NULL) == FNT_E_INVAL);
    EXPECT(fnt_cdc(x + 1, 64, &cp, NULL, NULL, NULL) == FNT_E_INVAL);
    EXPECT(fnt_cdc_long(x, 64, h, 66, 4, 0, NULL, NULL, NULL) == FNT_E_INVAL);
    EXPECT(fnt_cdc_long(x, 64, NULL, 10, 4, 0, NULL, NULL, NULL) == FNT_E_INVAL);
    h[5] = -33;
    EXPECT(fnt_cdc_long(x, 64, h, 10, 4, 0, NULL, NULL, NULL) == FNT_E_RANGE);
    h[5] = 0;
    EXPECT(fnt_cdc_long(x, 64, h, 10, 17, 0, NULL, NULL, NULL) == FNT_E_INVAL);
    EXPECT(fnt_aeq(x, 64, NULL, &ap, out, NULL) == FNT_E_INVAL);
    ap.out_shift = 25;
    EXPECT(fnt_aeq(x, 64, taps, &ap, out, NULL) == FNT_E_INVAL);
    ap.out_shift = 7;
    ap.const_unit = 0;
    EXPECT(fnt_aeq(x, 64, taps, &ap, out, NULL) == FNT_E_INVAL);
    ap.const_unit = 52;
    EXPECT(fnt_aeq(x, 64, taps, &ap, NULL, NULL) == FNT_E_INVAL);
    EXPECT(fnt_cdc_aeq(x, 64, NULL, taps, &ap, out, NULL) == FNT_E_INVAL);
    EXPECT(fnt_forward(NULL, NULL, 1, 4, 5, 0, NULL) != FNT_OK);
    EXPECT(fnt_forward((const uint32_t *)taps, (uint32_t *)out, 1, 9, 5, 0, NULL) != FNT_OK);
    EXPECT(fnt_plan_create(NULL, NULL, 0, NULL, NULL) == FNT_E_INVAL);
    EXPECT(fnt_plan_run(NULL, NULL) == FNT_E_INVAL);
    EXPECT(fnt_plan_run_graph(NULL, NULL) == FNT_E_INVAL);
    EXPECT(fnt_plan_get_info(NULL, NULL) == FNT_E_INVAL);
    EXPECT(fnt_plan_set_fused(NULL, 4, 0, 0) == FNT_E_INVAL);
    EXPECT(fnt_plan_destroy(NULL) == FNT_OK);
    EXPECT(fnt_session_create(NULL, NULL) == FNT_E_INVAL);
    EXPECT(fnt_session_destroy(NULL) == FNT_OK);
    EXPECT(fnt_cdc_aeq_batch_noalloc(NULL, FNT_NOALLOC_MAX_CHANNELS + 1, NULL) == FNT_E_INVAL);
    EXPECT(fnt_cdc_aeq_batch_noalloc(NULL, 3, NULL) == FNT_E_INVAL);
    EXPECT(strlen(fnt_last_error()) > 0);

    /* calls that reach the HIP runtime: with no GPU they must fail cleanly */
    fnt_channel_desc d;
    memset(&d, 0, sizeof d);
    d.in = x;
    d.out = out;
    d.taps = taps;
    d.n = 64;
    d.cdc = cp;
    d.aeq = ap;
    fnt_plan_config cfg = {0, 0, 1, 0, NULL};
    fnt_plan *plan = NULL;
    const int rc_plan = fnt_plan_create(&plan, &d, 1, &cfg, NULL);
    if (rc_plan == FNT_OK) {                 /* a GPU is present: run and tear down */
        fnt_plan_info info;
        EXPECT(fnt_plan_get_info(plan, &info) == FNT_OK && info.channels == 1);
        EXPECT(fnt_plan_destroy(plan) == FNT_OK);
    } else {
        EXPECT(plan == NULL);
        EXPECT(rc_plan == FNT_E_DEVICE || rc_plan == FNT_E_NOMEM);
    }
    fnt_session_config sc = {0, 16, 1u << 20, 0, 0, -1, 0};
    fnt_session *s = NULL;
    const int rc_s = fnt_session_create(&s, &sc);
    if (rc_s == FNT_OK) {
        fnt_session_stats st;
        EXPECT(fnt_session_get_stats(s, &st) == FNT_OK && st.submitted == 0);
        EXPECT(fnt_session_destroy(s) == FNT_OK);
    } else {
        EXPECT(s == NULL);
    }
    if (fails) return 1;
    printf("ok %d %d\n", rc_plan, rc_s);
    return 0;
}
